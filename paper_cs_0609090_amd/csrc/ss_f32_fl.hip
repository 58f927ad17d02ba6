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
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, gfx9 family
// Byte offset of the unused slots of a short row: every array of a chunk is
// below 2^31 bytes and a lane adds less than that, so the sum stays past the
// end of the buffer without wrapping: loads there return 0 and touch no
// memory, stores are dropped.
constexpr uint32_t kOutOfRange = 0x80000000u;

struct FlArgs {
    int32_t M, N, F, Fp, G;  // Fp = 64 * G frame lanes
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
};

__device__ __forceinline__ float norm_f(float m, float alpha, float beta) {
    const float v = __fsub_rn(__fmul_rn(alpha, m), beta);
    return v > 0.0f ? v : 0.0f;
}

// The code's index arrays are read-only for the whole call: reading them
// through the constant address space lets wave-uniform loads go to the
// scalar unit (s_load) instead of the vector memory path.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cptr(const T *p) {
    return (const __attribute__((address_space(4))) T *)(p);
}

// Buffer view of one frame-minor array: every access is a scalar element
// offset (SGPR) plus the lane's frame offset (one VGPR shared by all
// accesses), so no per-access 64-bit address is formed.
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ Buf(const void *p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3)) {}
    __device__ float ld(uint32_t lane_off, uint32_t elem_off) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, elem_off, 0));
    }
    __device__ void st(float v, uint32_t lane_off, uint32_t elem_off) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, lane_off, elem_off, 0);
    }
};

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
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u;             // lane offset in bytes
    const uint32_t rowb = (uint32_t)Fp * 4u;  // bytes per element row
    const Buf zb(zold, (uint32_t)a.N * rowb), lb(a.L, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    for (int m = r0; m < a.M; m += a.rwaves) {
        const int e0 = rp[m];
        const int d = rp[m + 1] - e0;
        float z[DMAX], t[DMAX];
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
            z[j] = zb.ld(fo, var[j]);
            if (UPDATE) t[j] = FIRST ? 0.0f : lb.ld(fo, pos[j]);
        }
        int syn = 0, par = 0;
        float min1 = INFINITY, min2 = INFINITY;
        int idx = 0;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const bool in = j < d;
            syn ^= (in && !(z[j] > 0.0f)) ? 1 : 0;
            if (UPDATE) {
                const float tj = __fsub_rn(z[j], t[j]);
                t[j] = tj;
                par ^= (in && tj < 0.0f) ? 1 : 0;
                const float av = in ? fabsf(tj) : INFINITY;
                min2 = fminf(min2, fmaxf(min1, av));
                idx = av < min1 ? j : idx;
                min1 = fminf(min1, av);
            }
        }
        if (syn_row >= 0 && syn) a.fail[(size_t)syn_row * Fp + f] = 1;
        if (UPDATE) {
            const float A = norm_f(min1, a.alpha, a.beta);
            const float B = norm_f(min2, a.alpha, a.beta);
            float out[DMAX];
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                const float mag = j == idx ? B : A;
                const bool neg = (par ^ (t[j] < 0.0f ? 1 : 0)) != 0;
                out[j] = neg ? -mag : mag;
            }
#pragma unroll
            for (int j = 0; j < DMAX; ++j) lb.st(out[j], fo, pos[j]);
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
    const uint32_t f = (uint32_t)(g * 64 + lane);
    const uint32_t fo = f * 4u;
    const uint32_t rowb = (uint32_t)Fp * 4u;
    const uint32_t nb = (uint32_t)a.N * rowb;
    const Buf zo(zold, nb), zn(znew, nb), z0(a.z0, nb), lb(a.L, a.ebytes);
    bool frozen = false;
    if (FREEZE) frozen = a.conv[f] != kNotConverged || a.fail[(size_t)fail_row * Fp + f] == 0;
    const auto *vp = cptr(a.vc_ptr);
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const uint32_t o = (uint32_t)n * rowb;
        if (FREEZE && frozen) {
            zn.st(zo.ld(fo, o), fo, o);
            continue;
        }
        const int e0 = vp[n], e1 = vp[n + 1];
        float s = z0.ld(fo, o);
        // eight messages per step, all loads in flight together; slots past
        // the variable's last edge are out of range and skipped (no +0.0 is
        // added, so the sum is exactly the ordered one)
        for (int e = e0; e < e1; e += 8) {
            float l[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) l[i] = lb.ld(fo, e + i < e1 ? (uint32_t)(e + i) * rowb : kOutOfRange);
#pragma unroll
            for (int i = 0; i < 8; ++i) s = e + i < e1 ? __fadd_rn(s, l[i]) : s;
        }
        zn.st(s, fo, o);
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

// Frames per call chunk: buffer offsets are 32-bit, so every frame-minor
// array of a chunk stays below 2 GiB (64-frame groups; 0 if even one group
// does not fit).
int fl_chunk_frames(int N, int64_t E) {
    const int64_t rowmax = std::max<int64_t>(E, N) * 4 * 64;  // bytes per element row of one group
    const int64_t groups = ((int64_t)0x7FFFFF00) / rowmax;      // arrays below 2^31 bytes
    return (int)std::min<int64_t>(groups * 64, (int64_t)1 << 30);
}

size_t fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter) {
    const int chunk = fl_chunk_frames(N, E);
    const int fr = std::min(n_frames, std::max(chunk, 1));
    const size_t Fp = (size_t)((fr + 63) / 64) * 64;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 3 * al((size_t)N * Fp * 4) + al((size_t)E * Fp * 4) + al((size_t)(max_iter + 1) * Fp * 4) + al(Fp * 4);
}

hipError_t launch_ss_f32_fl(const DecodeArgs &d, const int32_t *row_ptr, const uint32_t *row_ent, int64_t E,
                            int max_row_deg, int cu_count, hipStream_t s) {
    const int chunk = fl_chunk_frames(d.c.N, E);
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
        a.G = (F + 63) / 64;
        a.Fp = a.G * 64;
        a.alpha = d.alpha;
        a.beta = d.beta;
        a.row_ptr = row_ptr;
        a.row_ent = row_ent;
        a.vc_ptr = d.c.vc_ptr;
        const size_t Fp = (size_t)a.Fp;
        a.ebytes = (uint32_t)((size_t)E * Fp * 4);
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
        // about 32 wavefronts per CU, split over the frame groups; wavefronts with
        // an id past rwaves*G (the grid's rounding) return at once
        const int64_t want = (int64_t)std::max(cu_count, 1) * 32;
        a.rwaves = (int)std::max<int64_t>(1, std::min<int64_t>(want / a.G, std::max(a.M, a.N)));
        const unsigned grid = (unsigned)(((int64_t)a.rwaves * a.G + kWaves - 1) / kWaves);
        const int K = d.max_iter;
        hipError_t e;
        if (max_row_deg <= 8)
            e = run<8>(dc, a, K, grid, s);
        else if (max_row_deg <= 16)
            e = run<16>(dc, a, K, grid, s);
        else if (max_row_deg <= 32)
            e = run<32>(dc, a, K, grid, s);
        else
            e = run<64>(dc, a, K, grid, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ldpc
