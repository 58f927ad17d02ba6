// Learned normalised/offset min-sum (declared in include/ldpc_learn.h):
// forward and adjoint of the decoder unrolled over T iterations, with one
// (a, b) pair per iteration and check-degree class (the constant lambda and
// beta of Sec. III made per-iteration and per-class), in binary32 with
// frames across lanes (the layout of ss_f32_fl.hip: lane = frame,
// frame-minor arrays, messages in variable-major edge order).
//
//   forward   t_mn = Z^(t-1)_n - L^(t-1)_mn
//             L^(t)_mn = sgn * max(a[t,c] * min_{n' != n} |t_mn'| - b[t,c], 0)
//             Z^(t)_n  = Z^(0)_n + sum of L^(t) over M(n), ascending check order
//             loss_t   = sum_f sum_n softplus(s Z^(t)_n), s = 2x - 1
//   adjoint   Zbar^(t)_n = s sigma(s Z^(t)_n) + sum of tbar^(t+1) over M(n)
//             Lbar^(t)_mn = Zbar^(t)_n - tbar^(t+1)_mn
//             per row, with i1 / i2 the positions of the smallest / second
//             smallest |t| (lowest index on ties): every position j != i1 got
//             its magnitude from |t_i1|, position i1 from |t_i2|, so with
//             live_j = Lbar_j sgn_j [a m_j - b > 0]:
//               d/da += live_j m_j,  d/db -= live_j,
//               tbar_i1 = a sgn(t_i1) sum_{j != i1} live_j,
//               tbar_i2 = a sgn(t_i2) live_i1, other positions 0.
// Posteriors and messages are kept every `ckpt` iterations; the adjoint
// recomputes each segment forward from its checkpoint (the passes are
// deterministic, so the recomputed values equal the first ones bit for bit).
#include "../../include/ldpc_learn.h"
#include "code_handle.h"
#include "fl_common.h"

#include <cmath>
#include <string>
#include <vector>

namespace ldpc {
namespace {

using namespace fl;

constexpr int kMaxClasses = 8;

struct LrnArgs {
    int32_t M, N, F, Fp, G, rwaves, C, T;
    uint32_t ebytes, nbytes;  // bytes of one [E][Fp] / [N][Fp] float array
    const int32_t *row_ptr;
    const uint32_t *row_ent;  // [E + 64][2] {variable, variable-major position}
    const int32_t *vc_ptr;
    const int32_t *row_cls;   // [M] degree class of each row
    const float *W;           // [T][C][2] weights (a, b)
    const float *z0;          // [N][Fp]
    const uint8_t *tgt;       // [N][Fp] transmitted bits, or null (all-zero word)
};

__device__ __forceinline__ float softplus_f(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Check pass of iteration t (1-based): Lnew from zold and Lold (null: zeros).
template <int DMAX>
__global__ void __launch_bounds__(kBlock) lrn_check(LrnArgs a, const float *__restrict__ zold,
                                                    const float *__restrict__ Lold, float *__restrict__ Lnew,
                                                    int t) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u, rowb = (uint32_t)a.Fp * 4u;
    const Buf zb(zold, a.nbytes), lo(Lold ? Lold : Lnew, a.ebytes), ln(Lnew, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    const auto *rc = cptr(a.row_cls);
    const auto *Wt = cptr(a.W) + (size_t)(t - 1) * a.C * 2;
    for (int m = w / a.G; m < a.M; m += a.rwaves) {
        const int e0 = rp[m], d = rp[m + 1] - e0;
        const int c = rc[m];
        const float wa = Wt[2 * c], wb = Wt[2 * c + 1];
        uint32_t var[DMAX], pos[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t nv = re[2 * (e0 + j)], np = re[2 * (e0 + j) + 1];
            var[j] = j < d ? nv * rowb : kOutOfRange;
            pos[j] = j < d ? np * rowb : kOutOfRange;
        }
        float tt[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const float z = zb.ldf(fo, var[j]);
            tt[j] = Lold ? __fsub_rn(z, lo.ldf(fo, pos[j])) : z;
        }
        int par = 0, idx = 0;
        float min1 = INFINITY, min2 = INFINITY;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const bool in = j < d;
            par ^= (in && tt[j] < 0.0f) ? 1 : 0;
            const float av = in ? fabsf(tt[j]) : INFINITY;
            min2 = fminf(min2, fmaxf(min1, av));
            idx = av < min1 ? j : idx;
            min1 = fminf(min1, av);
        }
        const float v1 = __fsub_rn(__fmul_rn(wa, min1), wb), v2 = __fsub_rn(__fmul_rn(wa, min2), wb);
        const float A = v1 > 0.0f ? v1 : 0.0f, B = v2 > 0.0f ? v2 : 0.0f;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const float mag = j == idx ? B : A;
            ln.stf((par ^ (tt[j] < 0.0f ? 1 : 0)) ? -mag : mag, fo, pos[j]);
        }
    }
}

// Variable pass of iteration t: znew = z0 + sum of Lnew (ascending check
// order); adds sum softplus(s znew) into *loss.
__global__ void __launch_bounds__(kBlock) lrn_var(LrnArgs a, const float *__restrict__ Lnew, float *__restrict__ znew,
                                                  float *__restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u, rowb = (uint32_t)a.Fp * 4u;
    const Buf z0(a.z0, a.nbytes), zn(znew, a.nbytes), lb(Lnew, a.ebytes);
    const auto *vp = cptr(a.vc_ptr);
    const bool real = (int)f < a.F;
    float acc = 0.0f;
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const uint32_t o = (uint32_t)n * rowb;
        const int e0 = vp[n], e1 = vp[n + 1];
        float s = z0.ldf(fo, o);
        for (int e = e0; e < e1; e += 8) {
            float l[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) l[i] = lb.ldf(fo, e + i < e1 ? (uint32_t)(e + i) * rowb : kOutOfRange);
#pragma unroll
            for (int i = 0; i < 8; ++i) s = e + i < e1 ? __fadd_rn(s, l[i]) : s;
        }
        zn.stf(s, fo, o);
        const float sg = (a.tgt && a.tgt[(size_t)n * a.Fp + f]) ? 1.0f : -1.0f;
        if (real) acc += softplus_f(sg * s);
    }
    acc = wave_sum(acc);
    if (lane == 0) atomicAdd(loss, acc);
}

// Adjoint of the variable pass of iteration t: Zbar from the loss (weighted
// by lw, the objective's weight of iteration t) and from tbar (the extrinsic
// adjoints of iteration t+1, null at t = T); writes Lbar.
__global__ void __launch_bounds__(kBlock) lrn_var_bwd(LrnArgs a, const float *__restrict__ zt,
                                                      const float *__restrict__ tbar, float *__restrict__ Lbar,
                                                      float lw) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u, rowb = (uint32_t)a.Fp * 4u;
    const Buf zb(zt, a.nbytes), tb(tbar ? tbar : Lbar, a.ebytes), lbar(Lbar, a.ebytes);
    const auto *vp = cptr(a.vc_ptr);
    const bool real = (int)f < a.F;
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const uint32_t o = (uint32_t)n * rowb;
        const int e0 = vp[n], e1 = vp[n + 1];
        const float z = zb.ldf(fo, o);
        const float sg = (a.tgt && a.tgt[(size_t)n * a.Fp + f]) ? 1.0f : -1.0f;
        float zbar = real ? lw * (sg * sigmoid_f(sg * z)) : 0.0f;
        if (tbar) {
            for (int e = e0; e < e1; ++e) zbar += tb.ldf(fo, (uint32_t)e * rowb);
        }
        for (int e = e0; e < e1; ++e) {
            const uint32_t eo = (uint32_t)e * rowb;
            lbar.stf(tbar ? zbar - tb.ldf(fo, eo) : zbar, fo, eo);
        }
    }
}

// Adjoint of the check pass of iteration t: weight gradients into
// grad[t-1][c][0..1]; tbar (the adjoint of this iteration's extrinsics) when
// write_tbar.
template <int DMAX>
__global__ void __launch_bounds__(kBlock) lrn_check_bwd(LrnArgs a, const float *__restrict__ zold,
                                                        const float *__restrict__ Lold,
                                                        const float *__restrict__ Lbar, float *__restrict__ tbar,
                                                        float *__restrict__ grad, int t, int write_tbar) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u, rowb = (uint32_t)a.Fp * 4u;
    const Buf zb(zold, a.nbytes), lo(Lold ? Lold : Lbar, a.ebytes), lbar(Lbar, a.ebytes), tb(tbar, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    const auto *rc = cptr(a.row_cls);
    const auto *Wt = cptr(a.W) + (size_t)(t - 1) * a.C * 2;
    float ga[kMaxClasses], gb[kMaxClasses];
#pragma unroll
    for (int c = 0; c < kMaxClasses; ++c) ga[c] = gb[c] = 0.0f;
    for (int m = w / a.G; m < a.M; m += a.rwaves) {
        const int e0 = rp[m], d = rp[m + 1] - e0;
        const int c = rc[m];
        const float wa = Wt[2 * c], wb = Wt[2 * c + 1];
        uint32_t var[DMAX], pos[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t nv = re[2 * (e0 + j)], np = re[2 * (e0 + j) + 1];
            var[j] = j < d ? nv * rowb : kOutOfRange;
            pos[j] = j < d ? np * rowb : kOutOfRange;
        }
        float tt[DMAX], lb[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const float z = zb.ldf(fo, var[j]);
            tt[j] = Lold ? __fsub_rn(z, lo.ldf(fo, pos[j])) : z;
            lb[j] = lbar.ldf(fo, pos[j]);
        }
        int par = 0, i1 = 0, i2 = 0;
        float min1 = INFINITY, min2 = INFINITY;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const bool in = j < d;
            par ^= (in && tt[j] < 0.0f) ? 1 : 0;
            const float av = in ? fabsf(tt[j]) : INFINITY;
            if (av < min1) {
                min2 = min1;
                i2 = i1;
                min1 = av;
                i1 = j;
            } else if (av < min2) {
                min2 = av;
                i2 = j;
            }
        }
        const bool act1 = __fsub_rn(__fmul_rn(wa, min1), wb) > 0.0f;
        const bool act2 = __fsub_rn(__fmul_rn(wa, min2), wb) > 0.0f;
        float sum_other = 0.0f, live_i1 = 0.0f, da = 0.0f, db = 0.0f;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (j < d) {
                const bool neg = (par ^ (tt[j] < 0.0f ? 1 : 0)) != 0;
                const bool is1 = j == i1;
                const float live = (is1 ? act2 : act1) ? (neg ? -lb[j] : lb[j]) : 0.0f;
                da += live * (is1 ? min2 : min1);
                db -= live;
                if (is1)
                    live_i1 = live;
                else
                    sum_other += live;
            }
        }
#pragma unroll
        for (int cc = 0; cc < kMaxClasses; ++cc) {
            if (cc == c) {
                ga[cc] += da;
                gb[cc] += db;
            }
        }
        if (write_tbar) {
            float sgn1 = 1.0f, sgn2 = 1.0f;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j == i1) sgn1 = tt[j] < 0.0f ? -1.0f : 1.0f;
                if (j == i2) sgn2 = tt[j] < 0.0f ? -1.0f : 1.0f;
            }
            const float t1 = wa * sgn1 * sum_other, t2 = wa * sgn2 * live_i1;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) tb.stf(j == i1 ? t1 : (j == i2 ? t2 : 0.0f), fo, pos[j]);
        }
    }
    float *gt = grad + (size_t)(t - 1) * a.C * 2;
    for (int c = 0; c < a.C && c < kMaxClasses; ++c) {
        const float sa = wave_sum(ga[c]), sb = wave_sum(gb[c]);
        if (lane == 0) {
            atomicAdd(&gt[2 * c], sa);
            atomicAdd(&gt[2 * c + 1], sb);
        }
    }
}

__global__ void fill_zero(float *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Workspace: z0, target bits, Lbar, tbar, checkpoints (Z and L of
// iterations ckpt, 2 ckpt, ...), one segment of ckpt working slots and a
// scratch word.
struct Layout {
    size_t z0, tgt, lbar, tbar, cp, seg, scr, total;
    int ncp, nseg;
};

Layout layout_of(int N, int64_t E, int F, int T, int ckpt) {
    const size_t Fp = (size_t)((F + 63) / 64) * 64;
    const size_t zb = al256((size_t)N * Fp * 4), eb = al256((size_t)E * Fp * 4);
    Layout L{};
    L.ncp = T / ckpt;
    L.nseg = ckpt;
    size_t p = 0;
    L.z0 = p, p += zb;
    L.tgt = p, p += al256((size_t)N * Fp);
    L.lbar = p, p += eb;
    L.tbar = p, p += eb;
    L.cp = p, p += (size_t)L.ncp * (zb + eb);
    L.seg = p, p += (size_t)L.nseg * (zb + eb);
    L.scr = p, p += 256;  // loss sink of the adjoint's recomputations
    L.total = p;
    return L;
}

struct Ctx {
    LrnArgs a;
    Layout lay;
    uint8_t *ws;
    size_t zb, eb;
    int ckpt;
    unsigned grid;
    // buffers of iteration t: checkpoints at multiples of ckpt, else the
    // segment slot (t - 1) mod ckpt; t = 0: z0 and no messages
    float *Z(int t) const {
        if (t == 0) return const_cast<float *>(a.z0);
        if (t % ckpt == 0) return reinterpret_cast<float *>(ws + lay.cp + (size_t)(t / ckpt - 1) * (zb + eb));
        return reinterpret_cast<float *>(ws + lay.seg + (size_t)((t - 1) % ckpt) * (zb + eb));
    }
    float *Lm(int t) const {
        if (t == 0) return nullptr;
        return reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(Z(t)) + zb);
    }
};

ldpc_status make_ctx(const ldpc_code *c, int F, int T, int ckpt, const float *W, void *ws, size_t ws_bytes, Ctx *x) {
    if (!c || c->device < 0) return set_error(LDPC_EINVAL, "a device code handle is required");
    if (F <= 0 || T < 1 || ckpt < 1) return set_error(LDPC_EINVAL, "n_frames, T and ckpt must be >= 1");
    if (!W) return set_error(LDPC_EINVAL, "weights are required");
    if (c->learn_classes > kMaxClasses) return set_error(LDPC_EUNSUPPORTED, "more than 8 check-degree classes");
    if (c->D > 32) return set_error(LDPC_EUNSUPPORTED, "row degree above 32");
    if (ldpc::fl_chunk_frames(c->N, c->E) < F)
        return set_error(LDPC_EUNSUPPORTED, "batch too large for one frames-across-lanes chunk");
    x->lay = layout_of(c->N, c->E, F, T, ckpt);
    if (!ws || ws_bytes < x->lay.total) return set_error(LDPC_EINVAL, "workspace missing or too small");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return set_error(LDPC_EINVAL, "workspace must be 256-byte aligned");
    LrnArgs &a = x->a;
    a = LrnArgs{};
    a.M = c->M;
    a.N = c->N;
    a.F = F;
    a.G = (F + 63) / 64;
    a.Fp = a.G * 64;
    a.C = c->learn_classes;
    a.T = T;
    a.ebytes = (uint32_t)((size_t)c->E * a.Fp * 4);
    a.nbytes = (uint32_t)((size_t)c->N * a.Fp * 4);
    a.row_ptr = c->d_row_ptr;
    a.row_ent = c->d_row_ent;
    a.vc_ptr = c->d_vc_ptr;
    a.row_cls = c->d_row_cls;
    a.W = W;
    x->ws = static_cast<uint8_t *>(ws);
    a.z0 = reinterpret_cast<const float *>(x->ws + x->lay.z0);
    x->zb = al256((size_t)c->N * a.Fp * 4);
    x->eb = al256((size_t)c->E * a.Fp * 4);
    x->ckpt = ckpt;
    wave_layout(c->cu_count, a.G, std::max(a.M, a.N), &a.rwaves, &x->grid);
    return LDPC_OK;
}

template <int DMAX>
void forward_steps(const Ctx &x, int t_from, int t_to, float *loss, hipStream_t s) {
    // iterations t_from+1 .. t_to; loss (or null: recomputation, loss
    // discarded into a scratch word) per iteration
    for (int t = t_from + 1; t <= t_to; ++t) {
        hipLaunchKernelGGL((lrn_check<DMAX>), dim3(x.grid), dim3(kBlock), 0, s, x.a, x.Z(t - 1), x.Lm(t - 1),
                           x.Lm(t), t);
        hipLaunchKernelGGL(lrn_var, dim3(x.grid), dim3(kBlock), 0, s, x.a, x.Lm(t), x.Z(t),
                           loss ? loss + (t - 1) : reinterpret_cast<float *>(x.ws + x.lay.scr));
    }
}

// lw: host [T] weights of the iterations' losses in the objective, or null (all 1)
template <int DMAX>
void backward_all(const Ctx &x, float *grad, const float *lw, hipStream_t s) {
    const int T = x.a.T, k = x.ckpt;
    float *lbar = reinterpret_cast<float *>(x.ws + x.lay.lbar);
    float *tbar = reinterpret_cast<float *>(x.ws + x.lay.tbar);
    bool have_tbar = false;
    for (int t1 = T; t1 > 0;) {
        const int t0 = ((t1 - 1) / k) * k;  // segment (t0, t1]
        // recompute the segment's non-checkpoint iterations
        if (t1 - 1 > t0 || t1 % k != 0) {
            const int upto = (t1 % k == 0) ? t1 - 1 : t1;
            if (upto > t0) forward_steps<DMAX>(x, t0, upto, nullptr, s);
        }
        for (int t = t1; t > t0; --t) {
            hipLaunchKernelGGL(lrn_var_bwd, dim3(x.grid), dim3(kBlock), 0, s, x.a, x.Z(t),
                               have_tbar ? tbar : nullptr, lbar, lw ? lw[t - 1] : 1.0f);
            hipLaunchKernelGGL((lrn_check_bwd<DMAX>), dim3(x.grid), dim3(kBlock), 0, s, x.a, x.Z(t - 1),
                               x.Lm(t - 1), lbar, tbar, grad, t, t > 1 ? 1 : 0);
            have_tbar = true;
        }
        t1 = t0;
    }
}

}  // namespace
}  // namespace ldpc

using ldpc::set_error;

extern "C" {

ldpc_status ldpc_learn_workspace_size(const ldpc_code *code, int32_t n_frames, int32_t T, int32_t ckpt,
                                      size_t *bytes) {
    if (!code || !bytes) return set_error(LDPC_EINVAL, "NULL argument");
    if (n_frames < 1 || T < 1 || ckpt < 1) return set_error(LDPC_EINVAL, "n_frames, T and ckpt must be >= 1");
    *bytes = ldpc::layout_of(code->N, code->E, n_frames, T, ckpt).total;
    return LDPC_OK;
}

ldpc_status ldpc_learn_classes(const ldpc_code *code, int32_t *n_classes, int32_t *degrees) {
    if (!code || !n_classes) return set_error(LDPC_EINVAL, "NULL argument");
    *n_classes = code->learn_classes;
    if (degrees) std::copy(code->learn_degrees.begin(), code->learn_degrees.end(), degrees);
    return LDPC_OK;
}

ldpc_status ldpc_learn_forward(const ldpc_code *code, int32_t n_frames, const float *llr, const uint8_t *target,
                               int32_t T, const float *weights, int32_t ckpt, void *workspace,
                               size_t workspace_bytes, float *loss, float *post_out, void *stream) {
    ldpc::Ctx x;
    ldpc_status st = ldpc::make_ctx(code, n_frames, T, ckpt, weights, workspace, workspace_bytes, &x);
    if (st != LDPC_OK) return st;
    if (!llr || !loss) return set_error(LDPC_EINVAL, "llr and loss are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 tgrid((unsigned)((code->N + 63) / 64), (unsigned)x.a.G);
    hipLaunchKernelGGL(ldpc::fl::transpose_in<float>, tgrid, dim3(ldpc::fl::kBlock), 0, s, llr,
                       const_cast<float *>(x.a.z0), code->N, n_frames, x.a.Fp);
    if (target) {
        uint8_t *tg = x.ws + x.lay.tgt;
        hipLaunchKernelGGL(ldpc::fl::transpose_in<uint8_t>, tgrid, dim3(ldpc::fl::kBlock), 0, s, target, tg, code->N,
                           n_frames, x.a.Fp);
        x.a.tgt = tg;
    }
    hipLaunchKernelGGL(ldpc::fill_zero, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, loss, (int64_t)T);
    if (code->D <= 8)
        ldpc::forward_steps<8>(x, 0, T, loss, s);
    else if (code->D <= 16)
        ldpc::forward_steps<16>(x, 0, T, loss, s);
    else
        ldpc::forward_steps<32>(x, 0, T, loss, s);
    if (post_out) {
        // the hard decisions go to the scratch of the adjoint's extrinsics
        hipLaunchKernelGGL(ldpc::fl::transpose_out<float>, tgrid, dim3(ldpc::fl::kBlock), 0, s, x.Z(T), code->N,
                           n_frames, x.a.Fp, 1.0, x.ws + x.lay.tbar, post_out);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return LDPC_OK;
}

ldpc_status ldpc_learn_backward(const ldpc_code *code, int32_t n_frames, const uint8_t *target, int32_t T,
                                const float *weights, int32_t ckpt, void *workspace, size_t workspace_bytes,
                                float *grad, void *stream) {
    return ldpc_learn_backward_weighted(code, n_frames, target, T, weights, ckpt, workspace, workspace_bytes,
                                        nullptr, grad, stream);
}

ldpc_status ldpc_learn_backward_weighted(const ldpc_code *code, int32_t n_frames, const uint8_t *target,
                                         int32_t T, const float *weights, int32_t ckpt, void *workspace,
                                         size_t workspace_bytes, const float *loss_weights, float *grad,
                                         void *stream) {
    if (loss_weights && T > 0) {
        for (int t = 0; t < T; ++t)
            if (!std::isfinite(loss_weights[t]))
                return set_error(LDPC_EINVAL, "loss_weights must be finite");
    }
    ldpc::Ctx x;
    ldpc_status st = ldpc::make_ctx(code, n_frames, T, ckpt, weights, workspace, workspace_bytes, &x);
    if (st != LDPC_OK) return st;
    if (!grad) return set_error(LDPC_EINVAL, "grad is required");
    if (target) x.a.tgt = x.ws + x.lay.tgt;  // transposed by the forward call
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t ng = (int64_t)T * x.a.C * 2;
    hipLaunchKernelGGL(ldpc::fill_zero, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, grad, ng);
    if (code->D <= 8)
        ldpc::backward_all<8>(x, grad, loss_weights, s);
    else if (code->D <= 16)
        ldpc::backward_all<16>(x, grad, loss_weights, s);
    else
        ldpc::backward_all<32>(x, grad, loss_weights, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    return LDPC_OK;
}

}  // extern "C"
