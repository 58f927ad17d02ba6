// Two-scan (flooding) min-sum baseline, Sec. III: the schedule the single-scan
// form replaces.  One workgroup per frame.
//   horizontal scan, Eq. (1): per check row, from the stored variable-to-check
//     messages Z_mn (one per edge) compute and store L_mn (NMS/OMS applied);
//   vertical scan, Eq. (2): per variable, Z_n = Z^(0)_n + sum L_mn over M(n)
//     (ascending checks, through the variable-to-check index) and every Z_mn
//     written back: fixed point as sat(Z_n - L_mn) to +-31, which equals
//     saturating the exclusion sum of Eq. 2; binary32 as that exclusion sum
//     itself, Z^(0)_n + the other L_m'n in ascending check order.
// Per-edge state: Z_mn and L_mn, both int8 or binary32, [D][Mp] slot-major.
// The posterior array Z_n is kept for the hard decision and the output.
#include "ldpc_internal.h"

#include <type_traits>

namespace ldpc {
namespace {

template <typename T>
struct TS;

template <>
struct TS<int8_t> {
    using acc = int;
    using zn_t = int16_t;
    __device__ static int big() { return kQmax; }
    __device__ static int load_in(const void *p, size_t i) {
        const int v = static_cast<const int8_t *>(p)[i];
        return min(max(v, -kQmax), kQmax);
    }
    __device__ static int mag(int v) { return v < 0 ? -v : v; }
    __device__ static int norm(int m, const DecodeArgs &a) {
        const int v = ((m * a.a8 + 128) >> 8) - a.b_int;
        return v > 0 ? v : 0;
    }
    __device__ static int add(int x, int y) { return x + y; }
    __device__ static int ext(int s, int l) { return min(max(s - l, -kQmax), kQmax); }
    __device__ static float out(int z, const DecodeArgs &a) { return (float)((double)z * a.step); }
};

template <>
struct TS<float> {
    using acc = float;
    using zn_t = float;
    __device__ static float big() { return INFINITY; }
    __device__ static float load_in(const void *p, size_t i) { return static_cast<const float *>(p)[i]; }
    __device__ static float mag(float v) { return fabsf(v); }
    __device__ static float norm(float m, const DecodeArgs &a) {
        const float v = __fsub_rn(__fmul_rn(a.alpha, m), a.beta);
        return v > 0.0f ? v : 0.0f;
    }
    __device__ static float add(float x, float y) { return __fadd_rn(x, y); }
    __device__ static float ext(float s, float l) { return __fsub_rn(s, l); }
    __device__ static float out(float z, const DecodeArgs &) { return z; }
};

template <typename ZT>
__device__ void syndrome_pass_ts(int tid, int T, int Mp, int D, const uint32_t *__restrict__ ell,
                                 const ZT *Zn, int *flag) {
    for (int m = tid; m < Mp; m += T) {
        int p = 0;
        for (int j = 0; j < D; ++j) p ^= (Zn[ell[j * Mp + m]] > (ZT)0) ? 0 : 1;
        if (p) atomicOr(flag, 1);
    }
}

template <int DMAX, typename T, bool ML, bool ZL>
__global__ void __launch_bounds__(launch_bound_for(DMAX)) two_scan_kernel(DecodeArgs a) {
    using S = TS<T>;
    using A_t = typename S::acc;
    using ZN = typename S::zn_t;
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x;
    const int BT = blockDim.x;
    const int f = blockIdx.x;
    const int N = a.c.N, Mp = a.c.Mp, D = a.c.D;
    const int dummy = a.c.dummy;
    const uint32_t *__restrict__ ell = a.c.ell;
    const int32_t *__restrict__ vc_ptr = a.c.vc_ptr;
    const uint32_t *__restrict__ vc_slot = a.c.vc_slot;
    uint8_t *wsf = a.ws + (size_t)f * a.ws_stride;
    T *Zmn = ML ? reinterpret_cast<T *>(lds + a.off_msg) : reinterpret_cast<T *>(wsf + a.ws_off_msg);
    T *L = Zmn + (size_t)D * Mp;
    ZN *Zn = ZL ? reinterpret_cast<ZN *>(lds + a.off_z) : reinterpret_cast<ZN *>(wsf + a.ws_off_z);
    int *flag = reinterpret_cast<int *>(lds + a.off_aux);
    const size_t fo = (size_t)f * N;

    // Initialisation: Z^(0)_mn = Z^(0)_n (padding slots hold a value never selected)
    for (int i = tid; i < D * Mp; i += BT) {
        const uint32_t n = ell[i];
        Zmn[i] = (n != (uint32_t)dummy) ? (T)S::load_in(a.llr_in, fo + n) : (T)S::big();
    }
    for (int n = tid; n <= dummy; n += BT)
        Zn[n] = n < N ? (ZN)S::load_in(a.llr_in, fo + n) : (ZN)S::big();
    if (tid == 0) *flag = 0;
    __syncthreads();

    int iters = 0;
    bool converged = false;
    for (int k = 1; k <= a.max_iter; ++k) {
        // horizontal scan, Eq. (1)
        for (int m = tid; m < Mp; m += BT) {
            A_t tt[DMAX];
            A_t min1 = (A_t)S::big(), min2 = (A_t)S::big();
            int idx = 0;
            uint32_t par = 0;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const A_t t = (A_t)Zmn[j * Mp + m];
                    tt[j] = t;
                    par ^= (t < (A_t)0) ? 1u : 0u;
                    const A_t av = S::mag(t);
                    min2 = min(min2, max(min1, av));
                    idx = (av < min1) ? j : idx;
                    min1 = min(min1, av);
                }
            }
            const A_t Am = S::norm(min1, a);
            const A_t Bm = S::norm(min2, a);
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const A_t mag = (j == idx) ? Bm : Am;
                    const bool neg = (par ^ ((tt[j] < (A_t)0) ? 1u : 0u)) != 0u;
                    L[j * Mp + m] = (T)(neg ? -mag : mag);
                }
            }
        }
        __syncthreads();
        if (tid == 0) *flag = 0;
        // vertical scan, Eq. (2), and the posterior
        for (int n = tid; n < N; n += BT) {
            const int e0 = vc_ptr[n], e1 = vc_ptr[n + 1];
            A_t s = (A_t)S::load_in(a.llr_in, fo + n);
            for (int e = e0; e < e1; ++e) s = S::add(s, (A_t)L[vc_slot[e]]);
            Zn[n] = (ZN)s;
            for (int e = e0; e < e1; ++e) {
                const uint32_t slot = vc_slot[e];
                if constexpr (std::is_same<T, float>::value) {
                    A_t v = (A_t)S::load_in(a.llr_in, fo + n);
                    for (int e2 = e0; e2 < e1; ++e2)
                        if (e2 != e) v = S::add(v, (A_t)L[vc_slot[e2]]);
                    Zmn[slot] = (T)v;
                } else {
                    Zmn[slot] = (T)S::ext(s, (A_t)L[slot]);
                }
            }
        }
        __syncthreads();
        iters = k;
        if (a.early_stop) {
            syndrome_pass_ts<ZN>(tid, BT, Mp, D, ell, Zn, flag);
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
        syndrome_pass_ts<ZN>(tid, BT, Mp, D, ell, Zn, flag);
        __syncthreads();
        ok = (*flag == 0);
    }
    for (int n = tid; n < N; n += BT) {
        const A_t z = (A_t)Zn[n];
        a.hard_out[fo + n] = z > (A_t)0 ? 0 : 1;
        if (a.llr_out) a.llr_out[fo + n] = S::out(z, a);
    }
    if (tid == 0) {
        a.iters_out[f] = iters;
        a.ok_out[f] = (uint8_t)ok;
    }
}

template <int DMAX, typename T, bool ML, bool ZL>
hipError_t launch_one(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    auto kern = two_scan_kernel<DMAX, T, ML, ZL>;
    if (c.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_frames), dim3((unsigned)c.threads), c.lds, s, a);
    return hipGetLastError();
}

template <int DMAX, typename T>
hipError_t launch_t(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    if (c.msg_lds && c.z_lds) return launch_one<DMAX, T, true, true>(a, c, s);
    if (!c.msg_lds && c.z_lds) return launch_one<DMAX, T, false, true>(a, c, s);
    if (!c.msg_lds && !c.z_lds) return launch_one<DMAX, T, false, false>(a, c, s);
    return hipErrorInvalidValue;
}

template <int DMAX>
hipError_t launch_dmax(const DecodeArgs &a, int msg, const LaunchCfg &c, hipStream_t s) {
    return msg == MSG_INT8 ? launch_t<DMAX, int8_t>(a, c, s) : launch_t<DMAX, float>(a, c, s);
}

}  // namespace

hipError_t launch_two_scan(const DecodeArgs &a, int msg, const LaunchCfg &c, hipStream_t s) {
    switch (c.dmax) {
        case 8: return launch_dmax<8>(a, msg, c, s);
        case 16: return launch_dmax<16>(a, msg, c, s);
        case 32: return launch_dmax<32>(a, msg, c, s);
        case 64: return launch_dmax<64>(a, msg, c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpc
