// Single-scan min-sum in binary32 (Sec. IV, Eq. 3), one workgroup per frame.
//
// Check pass (one row per thread, check-to-variable addressing only):
//   t_j = Z^(k-1)[n_j] - L^(k-1)_j, min1/argmin/min2 of |t_j|, sign parity,
//   A = max(alpha*min1 - beta, 0), B = max(alpha*min2 - beta, 0) (the product
//   rounded before the subtraction), L^(k)_j = sign_j * (j == argmin ? B : A).
// Variable pass: Z^(k)[n] = Z^(0)[n] + sum of the new L over M(n), added in
// ascending check order.  Floating-point addition is not associative, so the
// sum is gathered in that fixed order instead of being scattered with atomics:
// the result is deterministic and reproduces a sequential decoder that visits
// the checks in row order.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

__device__ __forceinline__ float norm_f(float m, float alpha, float beta) {
    const float v = __fsub_rn(__fmul_rn(alpha, m), beta);
    return v > 0.0f ? v : 0.0f;
}

__device__ void syndrome_pass_f(int tid, int T, int Mp, int D, const uint32_t *__restrict__ ell,
                                const float *Z, int *flag) {
    for (int m = tid; m < Mp; m += T) {
        int p = 0;
        for (int j = 0; j < D; ++j) p ^= (Z[ell[j * Mp + m]] > 0.0f) ? 0 : 1;
        if (p) atomicOr(flag, 1);
    }
}

template <int DMAX, bool ML, bool ZL>
__global__ void __launch_bounds__(launch_bound_for(DMAX)) ss_f32_kernel(DecodeArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const int f = blockIdx.x;
    const int N = a.c.N, Mp = a.c.Mp, D = a.c.D;
    const int dummy = a.c.dummy;
    const uint32_t *__restrict__ ell = a.c.ell;
    const int32_t *__restrict__ vc_ptr = a.c.vc_ptr;
    const uint32_t *__restrict__ vc_slot = a.c.vc_slot;
    uint8_t *wsf = a.ws + (size_t)f * a.ws_stride;
    float *Z = ZL ? reinterpret_cast<float *>(lds + a.off_z) : reinterpret_cast<float *>(wsf + a.ws_off_z);
    float *L = ML ? reinterpret_cast<float *>(lds + a.off_msg) : reinterpret_cast<float *>(wsf + a.ws_off_msg);
    int *flag = reinterpret_cast<int *>(lds + a.off_aux);
    const float *__restrict__ z0 = static_cast<const float *>(a.llr_in) + (size_t)f * N;
    const float alpha = a.alpha, beta = a.beta;

    for (int n = tid; n <= dummy; n += T) Z[n] = n < N ? z0[n] : (n == dummy ? INFINITY : 0.0f);
    for (int i = tid; i < D * Mp; i += T) L[i] = 0.0f;
    if (tid == 0) *flag = 0;
    __syncthreads();

    int iters = 0;
    bool converged = false;
    for (int k = 1; k <= a.max_iter; ++k) {
        for (int m = tid; m < Mp; m += T) {
            float tt[DMAX];
            float min1 = INFINITY, min2 = INFINITY;
            int idx = 0;
            uint32_t par = 0;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const uint32_t n = ell[j * Mp + m];
                    const float t = __fsub_rn(Z[n], L[j * Mp + m]);
                    tt[j] = t;
                    par ^= (t < 0.0f) ? 1u : 0u;
                    const float av = fabsf(t);
                    min2 = fminf(min2, fmaxf(min1, av));
                    idx = (av < min1) ? j : idx;
                    min1 = fminf(min1, av);
                }
            }
            const float A = norm_f(min1, alpha, beta);
            const float B = norm_f(min2, alpha, beta);
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const float mag = (j == idx) ? B : A;
                    const bool neg = (par ^ ((tt[j] < 0.0f) ? 1u : 0u)) != 0u;
                    L[j * Mp + m] = neg ? -mag : mag;
                }
            }
        }
        __syncthreads();
        if (tid == 0) *flag = 0;
        for (int n = tid; n < N; n += T) {
            float s = z0[n];
            const int e1 = vc_ptr[n + 1];
            for (int e = vc_ptr[n]; e < e1; ++e) s = __fadd_rn(s, L[vc_slot[e]]);
            Z[n] = s;
        }
        __syncthreads();
        iters = k;
        if (a.early_stop) {
            syndrome_pass_f(tid, T, Mp, D, ell, Z, flag);
            __syncthreads();
            if (*flag == 0) {
                converged = true;
                break;
            }
        }
    }
    int ok = 1;
    if (!converged) {
        __syncthreads();
        if (tid == 0) *flag = 0;
        __syncthreads();
        syndrome_pass_f(tid, T, Mp, D, ell, Z, flag);
        __syncthreads();
        ok = (*flag == 0);
    }
    for (int n = tid; n < N; n += T) {
        const float z = Z[n];
        a.hard_out[(size_t)f * N + n] = z > 0.0f ? 0 : 1;
        if (a.llr_out) a.llr_out[(size_t)f * N + n] = z;
    }
    if (tid == 0) {
        a.iters_out[f] = iters;
        a.ok_out[f] = (uint8_t)ok;
    }
}

template <int DMAX, bool ML, bool ZL>
hipError_t launch_one(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    auto kern = ss_f32_kernel<DMAX, ML, ZL>;
    if (c.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_frames), dim3((unsigned)c.threads), c.lds, s, a);
    return hipGetLastError();
}

template <int DMAX>
hipError_t launch_dmax(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    if (c.msg_lds && c.z_lds) return launch_one<DMAX, true, true>(a, c, s);
    if (!c.msg_lds && c.z_lds) return launch_one<DMAX, false, true>(a, c, s);
    if (!c.msg_lds && !c.z_lds) return launch_one<DMAX, false, false>(a, c, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ss_f32(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    switch (c.dmax) {
        case 8: return launch_dmax<8>(a, c, s);
        case 16: return launch_dmax<16>(a, c, s);
        case 32: return launch_dmax<32>(a, c, s);
        case 64: return launch_dmax<64>(a, c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpc
