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
#include "ldpc_internal.h"

#include <algorithm>
#include <climits>

namespace ldpc {
namespace {

constexpr int kWaves = 4;  // wavefronts per workgroup
constexpr int kBlock = 64 * kWaves;
constexpr int kNotConverged = INT_MAX;

struct FlArgs {
    int32_t M, N, F, Fp, G;  // Fp = 64 * G frame lanes
    int32_t rwaves;          // wavefronts per frame group in the strided passes
    float alpha, beta;
    const int32_t *row_ptr;  // [M+1]
    const uint2 *row_ent;    // [E] per check-to-variable edge: {variable, message position}
    const int32_t *vc_ptr;   // [N+1] message positions of variable n: vc_ptr[n] .. vc_ptr[n+1]
    float *z0;               // [N][Fp]
    float *zbuf[2];          // [N][Fp] posteriors of odd / even iterations
    float *L;                // [E][Fp] messages, variable-major edge order
    int32_t *fail;           // [K+1][Fp] 1 = syndrome of Z^(k) not satisfied
    int32_t *conv;           // [Fp] first iteration whose syndrome passed
};

__device__ __forceinline__ float norm_f(float m, float alpha, float beta) {
    const float v = __fsub_rn(__fmul_rn(alpha, m), beta);
    return v > 0.0f ? v : 0.0f;
}

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWaves + (threadIdx.x >> 6)));
}

// llr_in [F][N] -> z0 [N][Fp] (frames >= F read as 0), 64x64 tiles via LDS.
__global__ void __launch_bounds__(kBlock) fl_transpose_in(const float *__restrict__ in, float *__restrict__ z0,
                                                          int N, int F, int Fp) {
    __shared__ float tile[64][65];
    const int n0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += kWaves) {
        const int f = f0 + r, n = n0 + tx;
        tile[r][tx] = (f < F && n < N) ? in[(size_t)f * N + n] : 0.0f;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += kWaves) {
        const int n = n0 + r, f = f0 + tx;
        if (n < N) z0[(size_t)n * Fp + f] = tile[tx][r];
    }
}

__global__ void __launch_bounds__(kBlock) fl_init_flags(int32_t *fail, int64_t nfail, int32_t *conv, int Fp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nfail) fail[i] = 0;
    if (i < Fp) conv[i] = kNotConverged;
}

// Check pass of iteration k (UPDATE), or the syndrome of zold alone.
//   syn_row >= 0: record rows failing the syndrome of zold in fail[syn_row]
//   conv_k  >= 1: first fold fail[conv_k] into conv (one wavefront)
// FIRST: L^(k-1) = 0 (iteration 1), the message array is not read.
template <int DMAX, bool UPDATE, bool FIRST>
__global__ void __launch_bounds__(kBlock) fl_check(FlArgs a, const float *__restrict__ zold, int syn_row,
                                                   int conv_k) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (conv_k >= 1 && w == 0) {
        for (int f = lane; f < Fp; f += 64) {
            const int c = a.conv[f];
            if (c == kNotConverged && a.fail[(size_t)conv_k * Fp + f] == 0) a.conv[f] = conv_k;
        }
    }
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const int r0 = w / a.G;
    const int f = g * 64 + lane;
    for (int m = r0; m < a.M; m += a.rwaves) {
        const int e0 = a.row_ptr[m];
        const int d = a.row_ptr[m + 1] - e0;
        float z[DMAX], t[DMAX];
        uint32_t pos[DMAX];
        // all loads of the row first, then the arithmetic
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (j < d) {
                const uint2 ent = a.row_ent[e0 + j];
                pos[j] = ent.y;
                z[j] = zold[(size_t)ent.x * Fp + f];
                if (UPDATE) t[j] = FIRST ? 0.0f : a.L[(size_t)ent.y * Fp + f];
            }
        }
        int syn = 0, par = 0;
        float min1 = INFINITY, min2 = INFINITY;
        int idx = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (j < d) {
                syn ^= z[j] > 0.0f ? 0 : 1;
                if (UPDATE) {
                    const float tj = __fsub_rn(z[j], t[j]);
                    t[j] = tj;
                    par ^= tj < 0.0f ? 1 : 0;
                    const float av = fabsf(tj);
                    min2 = fminf(min2, fmaxf(min1, av));
                    idx = av < min1 ? j : idx;
                    min1 = fminf(min1, av);
                }
            }
        }
        if (syn_row >= 0 && syn) a.fail[(size_t)syn_row * Fp + f] = 1;
        if (UPDATE) {
            const float A = norm_f(min1, a.alpha, a.beta);
            const float B = norm_f(min2, a.alpha, a.beta);
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < d) {
                    const float mag = j == idx ? B : A;
                    const bool neg = (par ^ (t[j] < 0.0f ? 1 : 0)) != 0;
                    a.L[(size_t)pos[j] * Fp + f] = neg ? -mag : mag;
                }
            }
        }
    }
}

// Variable pass of iteration k: znew = z0 + messages in ascending check
// order; frames frozen by the early stop copy zold instead.
template <bool FREEZE>
__global__ void __launch_bounds__(kBlock) fl_var(FlArgs a, const float *__restrict__ zold, float *__restrict__ znew,
                                                 int fail_row) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const int f = g * 64 + lane;
    bool frozen = false;
    if (FREEZE) frozen = a.conv[f] != kNotConverged || a.fail[(size_t)fail_row * Fp + f] == 0;
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const size_t o = (size_t)n * Fp + f;
        if (FREEZE && frozen) {
            znew[o] = zold[o];
            continue;
        }
        const int e0 = a.vc_ptr[n], e1 = a.vc_ptr[n + 1];
        float s = a.z0[o];
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
            const float l0 = a.L[(size_t)e * Fp + f];
            const float l1 = a.L[(size_t)(e + 1) * Fp + f];
            const float l2 = a.L[(size_t)(e + 2) * Fp + f];
            const float l3 = a.L[(size_t)(e + 3) * Fp + f];
            s = __fadd_rn(__fadd_rn(__fadd_rn(__fadd_rn(s, l0), l1), l2), l3);
        }
        for (; e < e1; ++e) s = __fadd_rn(s, a.L[(size_t)e * Fp + f]);
        znew[o] = s;
    }
}

// Per-frame results: iterations and syndrome flag.
__global__ void __launch_bounds__(kBlock) fl_frame_out(FlArgs a, int K, int early_stop, int32_t *__restrict__ iters,
                                                       uint8_t *__restrict__ ok) {
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= a.F) return;
    const int Fp = a.Fp;
    int it = K;
    if (early_stop) {
        int c = a.conv[f];
        for (int k = (K >= 2 ? K - 1 : 1); k <= K && c == kNotConverged; ++k)
            if (a.fail[(size_t)k * Fp + f] == 0) c = k;
        if (c != kNotConverged) it = c;
    }
    iters[f] = it;
    ok[f] = a.fail[(size_t)K * Fp + f] == 0 ? 1 : 0;
}

// z [N][Fp] -> hard [F][N] (and llr [F][N]), 64x64 tiles via LDS.
__global__ void __launch_bounds__(kBlock) fl_transpose_out(const float *__restrict__ z, int N, int F, int Fp,
                                                           uint8_t *__restrict__ hard, float *__restrict__ llr) {
    __shared__ float tile[64][65];
    const int n0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += kWaves) {
        const int n = n0 + r;
        tile[r][tx] = n < N ? z[(size_t)n * Fp + f0 + tx] : 0.0f;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += kWaves) {
        const int f = f0 + r, n = n0 + tx;
        if (f < F && n < N) {
            const float v = tile[tx][r];
            hard[(size_t)f * N + n] = v > 0.0f ? 0 : 1;
            if (llr) llr[(size_t)f * N + n] = v;
        }
    }
}

template <int DMAX>
hipError_t run(const DecodeArgs &d, const FlArgs &a, int K, unsigned grid, hipStream_t s) {
    const bool es = d.early_stop != 0;
    const dim3 tgrid((unsigned)((a.N + 63) / 64), (unsigned)a.G);
    hipLaunchKernelGGL(fl_transpose_in, tgrid, dim3(kBlock), 0, s, static_cast<const float *>(d.llr_in), a.z0,
                       a.N, a.F, a.Fp);
    const int64_t nfail = (int64_t)(K + 1) * a.Fp;
    hipLaunchKernelGGL(fl_init_flags, dim3((unsigned)((std::max<int64_t>(nfail, a.Fp) + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a.fail, nfail, a.conv, a.Fp);
    const float *zold = a.z0;
    for (int k = 1; k <= K; ++k) {
        float *znew = a.zbuf[k & 1];
        // syndrome of Z^(k-1) (k >= 2), fold fail[k-2] into conv (k >= 3)
        const int syn_row = (es && k >= 2) ? k - 1 : -1;
        const int conv_k = (es && k >= 3) ? k - 2 : 0;
        if (k == 1)
            hipLaunchKernelGGL((fl_check<DMAX, true, true>), dim3(grid), dim3(kBlock), 0, s, a, zold, syn_row,
                               conv_k);
        else
            hipLaunchKernelGGL((fl_check<DMAX, true, false>), dim3(grid), dim3(kBlock), 0, s, a, zold, syn_row,
                               conv_k);
        if (es && k >= 2)
            hipLaunchKernelGGL(fl_var<true>, dim3(grid), dim3(kBlock), 0, s, a, zold, znew, k - 1);
        else
            hipLaunchKernelGGL(fl_var<false>, dim3(grid), dim3(kBlock), 0, s, a, zold, znew, 0);
        zold = znew;
    }
    // syndrome of the final posteriors, then the outputs
    hipLaunchKernelGGL((fl_check<DMAX, false, false>), dim3(grid), dim3(kBlock), 0, s, a, zold, K,
                       (es && K >= 3) ? K - 2 : 0);
    hipLaunchKernelGGL(fl_frame_out, dim3((unsigned)((a.F + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, K,
                       d.early_stop, d.iters_out, d.ok_out);
    hipLaunchKernelGGL(fl_transpose_out, tgrid, dim3(kBlock), 0, s, zold, a.N, a.F, a.Fp, d.hard_out, d.llr_out);
    return hipGetLastError();
}

}  // namespace

size_t fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter) {
    const size_t Fp = (size_t)((n_frames + 63) / 64) * 64;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 3 * al((size_t)N * Fp * 4) + al((size_t)E * Fp * 4) + al((size_t)(max_iter + 1) * Fp * 4) + al(Fp * 4);
}

hipError_t launch_ss_f32_fl(const DecodeArgs &d, const int32_t *row_ptr, const uint2 *row_ent, int64_t E,
                            int max_row_deg, int cu_count, hipStream_t s) {
    FlArgs a{};
    a.M = d.c.M;
    a.N = d.c.N;
    a.F = d.n_frames;
    a.G = (d.n_frames + 63) / 64;
    a.Fp = a.G * 64;
    a.alpha = d.alpha;
    a.beta = d.beta;
    a.row_ptr = row_ptr;
    a.row_ent = row_ent;
    a.vc_ptr = d.c.vc_ptr;
    const size_t Fp = (size_t)a.Fp;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    uint8_t *p = d.ws;
    a.z0 = reinterpret_cast<float *>(p);
    p += al((size_t)a.N * Fp * 4);
    a.zbuf[0] = reinterpret_cast<float *>(p);
    p += al((size_t)a.N * Fp * 4);
    a.zbuf[1] = reinterpret_cast<float *>(p);
    p += al((size_t)a.N * Fp * 4);
    a.L = reinterpret_cast<float *>(p);
    p += al((size_t)E * Fp * 4);
    a.fail = reinterpret_cast<int32_t *>(p);
    p += al((size_t)(d.max_iter + 1) * Fp * 4);
    a.conv = reinterpret_cast<int32_t *>(p);
    // about 16 wavefronts per CU, split over the frame groups; wavefronts with
    // an id past rwaves*G (the grid's rounding) return at once
    const int64_t want = (int64_t)std::max(cu_count, 1) * 16;
    a.rwaves = (int)std::max<int64_t>(1, std::min<int64_t>(want / a.G, std::max(a.M, a.N)));
    const unsigned grid = (unsigned)(((int64_t)a.rwaves * a.G + kWaves - 1) / kWaves);
    const int K = d.max_iter;
    if (max_row_deg <= 8) return run<8>(d, a, K, grid, s);
    if (max_row_deg <= 16) return run<16>(d, a, K, grid, s);
    if (max_row_deg <= 32) return run<32>(d, a, K, grid, s);
    if (max_row_deg <= 64) return run<64>(d, a, K, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace ldpc
