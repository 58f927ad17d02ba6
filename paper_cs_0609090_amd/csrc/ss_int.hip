// Single-scan min-sum in b-bit fixed point: int8 messages (Sec. IV, Eq. 3;
// b = 6, 7 or 8) and the compressed 1-bit form (Sec. V, 6-bit values), one
// workgroup per frame.  Below, 31 and 62 are the 6-bit Q and 2Q; b-bit
// messages use Q = 2^(b-1) - 1 and 2Q in their place, with Z_old in int16
// for b = 8.
//
// Per frame and iteration k the workgroup makes one pass over the
// check-to-variable addressing (slot-major ELL, a thread per check row):
//   t_j   = sat31(Z^(k-1)[n_j] - L^(k-1)_j)                 (Eq. 3, extrinsic)
//   min1/argmin/min2 of |t_j| and the XOR of the sign bits  (row reduction)
//   A = norm(min1), B = norm(min2)                           (Sec. III NMS/OMS)
//   L^(k)_j = sign_j * (j == argmin ? B : A)
//   Z_acc[n_j] += L^(k)_j - L^(k-1)_j                        (LDS atomic add)
// so Z_acc always equals Z^(0) + sum_m L_mn (integer sums are exact, so the
// order of the atomics does not matter).  A second, per-variable pass copies
// Z_acc into the gather array Z_old saturated to +-62: for any |L| <= 31,
// sat31(sat62(Z) - L) == sat31(Z - L), so one byte per variable is enough for
// the extrinsic and for the hard decision (Z <= 0 <=> sat62(Z) <= 0).
//
// LDS per frame: Z_old (1 byte/variable) + Z_acc (zpack fields per 32-bit
// word, each biased so partial sums never leave the field: a negative delta
// shifted into its field then never borrows from a neighbour) + optionally the
// message state.  Message state:
//   INT8  int8 L[D][Mp]
//   1BIT  uint64 sign words [D][Mp/64] (bit = lane of the wavefront, written
//         with a ballot) + uint16 state[Mp] = A | B << 5 | n~ << 10.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

struct ZPack {
    int P;
    int bits;
    uint32_t mask;
    int bias;
};

__device__ __forceinline__ ZPack zpack_of(int P) {
    ZPack z;
    z.P = P;
    z.bits = (P == 1) ? 32 : (P == 2 ? 16 : 10);
    z.mask = (P == 1) ? 0xFFFFFFFFu : ((1u << z.bits) - 1u);
    z.bias = (P == 1) ? 0 : (1 << (z.bits - 1));
    return z;
}

// word index and bit shift of variable n's accumulator field
__device__ __forceinline__ void zloc(uint32_t n, int P, uint32_t &word, uint32_t &shift) {
    if (P == 1) {
        word = n;
        shift = 0;
    } else if (P == 2) {
        word = n >> 1;
        shift = (n & 1u) << 4;
    } else {
        word = __umulhi(n, 0xAAAAAAABu) >> 1;  // n / 3
        shift = (n - word * 3u) * 10u;
    }
}

__device__ __forceinline__ int zfield(uint32_t v, uint32_t shift, const ZPack &z) {
    if (z.P == 1) return (int)v;
    return (int)((v >> shift) & z.mask) - z.bias;
}

__device__ __forceinline__ int clamp_i(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ int norm_q(int mag, int a8, int b) {
    const int v = ((mag * a8 + 128) >> 8) - b;
    return v > 0 ? v : 0;
}

// Row parity of hard decisions; sets *flag when a check fails.
template <typename ZT>
__device__ void syndrome_pass(int tid, int T, int Mp, int D, const uint32_t *__restrict__ ell,
                              const ZT *zold, int *flag) {
    for (int m = tid; m < Mp; m += T) {
        int p = 0;
        for (int j = 0; j < D; ++j) p ^= (zold[ell[j * Mp + m]] <= 0) ? 1 : 0;
        if (p) atomicOr(flag, 1);
    }
}

// FUSED (early stop, hard decisions only): the syndrome of the hard
// decisions of Z^(k-1) is formed from the Z_old gathers of iteration k; a
// zero syndrome stops the frame with k-1 iterations, its decisions read from
// Z_old (the saturated copy keeps the sign and zero of Z^(k-1)).  Otherwise a
// separate check pass follows each iteration.
// b-bit messages: extrinsics saturate to Q = a.qmax, the stored Z_old to
// 2Q = a.zmax, held in ZT (int8 up to 7 bits, int16 for 8).
template <int DMAX, int MSG, bool MSG_LDS, bool FUSED, typename ZT>
__global__ void __launch_bounds__(launch_bound_for(DMAX)) ss_int_kernel(DecodeArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const int f = blockIdx.x;
    const int N = a.c.N, Mp = a.c.Mp, D = a.c.D;
    const uint32_t dummy = (uint32_t)a.c.dummy;
    const uint32_t *__restrict__ ell = a.c.ell;
    ZT *zold = reinterpret_cast<ZT *>(lds + a.off_zold);
    const int Q = a.qmax, Z2 = a.zmax;
    uint32_t *zacc = reinterpret_cast<uint32_t *>(lds + a.off_zacc);
    int *flag = reinterpret_cast<int *>(lds + a.off_aux);  // [0]: separate check, [1], [2]: fused
    uint8_t *st = MSG_LDS ? (lds + a.off_msg) : (a.ws + (size_t)f * a.ws_stride + a.ws_off_msg);
    const int8_t *__restrict__ z0 = static_cast<const int8_t *>(a.llr_in) + (size_t)f * N;
    const int P = a.zpack;
    const ZPack zp = zpack_of(P);
    const int nwords = (int)(dummy / (uint32_t)P) + 1;
    const int MpW = Mp >> 6;  // sign words per slot (1BIT)

    // ---- initialisation: Z_acc = Z_old = Z^(0), L^(0) = 0 (1BIT: A = B = n~ = 0, s = 0)
    for (int w = tid; w < nwords; w += T) {
        uint32_t v = 0;
        for (int i = 0; i < P; ++i) {
            const int n = w * P + i;
            const int z = n < N ? clamp_i(z0[n], -Q, Q) : 0;
            v |= (uint32_t)(z + zp.bias) << (i * zp.bits);
        }
        zacc[w] = v;
    }
    for (int n = tid; n <= (int)dummy; n += T)
        zold[n] = (ZT)(n < N ? clamp_i(z0[n], -Q, Q) : (n == (int)dummy ? Z2 : 0));
    {
        const int words = (MSG == MSG_INT8) ? (D * Mp) / 4 : (D * MpW * 8 + 2 * Mp) / 4;
        uint32_t *s32 = reinterpret_cast<uint32_t *>(st);
        for (int i = tid; i < words; i += T) s32[i] = 0u;
    }
    if (tid == 0) {
        flag[0] = 0;
        flag[1] = 0;
        flag[2] = 0;
    }
    __syncthreads();

    int8_t *L8 = reinterpret_cast<int8_t *>(st);
    unsigned long long *sgn = reinterpret_cast<unsigned long long *>(st);
    uint16_t *cst = reinterpret_cast<uint16_t *>(st + (size_t)D * MpW * 8);

    int a8 = a.a8, bq = a.b_int;  // normalisation pair
    int iters = 0;
    bool converged = false;  // the decision of the last completed iteration is a codeword
    bool conv_prev = false;  // FUSED: that of the iteration before the last one is
    for (int k = 1; k <= a.max_iter; ++k) {
        // FUSED: the sign bit collects odd hard-decision parities of Z^(k-1)
        // rows; flag[1 + (k & 1)] is set by this iteration and read after its
        // first barrier, the other one (read last iteration) is cleared here
        int zodd = 0;
        if (FUSED && tid == 0) flag[1 + ((k + 1) & 1)] = 0;
        if (a.wsched) sched_pair(a, k, a8, bq);  // per-iteration pair (Sec. III's lambda_k, beta_k)
        // ---- check pass (Eq. 3), one row per thread
        for (int m = tid; m < Mp; m += T) {
            uint32_t nid[DMAX];
            int tt[DMAX];
            int lo[DMAX];
            uint32_t min1 = 0xFFFFFFFFu, min2 = 0xFFFFFFFFu;
            int par = 0, hpar = 0;
            int Ao = 0, Bo = 0, Io = 0;
            if (MSG == MSG_1BIT) {
                const uint32_t s = cst[m];
                Ao = s & 31u;
                Bo = (s >> 5) & 31u;
                Io = s >> 10;
            }
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const uint32_t n = ell[j * Mp + m];
                    nid[j] = n;
                    int l;
                    if (MSG == MSG_INT8) {
                        l = L8[j * Mp + m];
                    } else {  // L^(k-1) = s f(A, B, n, n~)
                        const unsigned long long wbits = sgn[j * MpW + (m >> 6)];
                        const int fv = (j == Io) ? Bo : Ao;
                        l = ((wbits >> (m & 63)) & 1ull) ? -fv : fv;
                    }
                    lo[j] = l;
                    const int zv = (int)zold[n];
                    if (FUSED) hpar ^= zv - 1;  // sign bit: Z_old <= 0
                    const int t = clamp_i(zv - l, -Q, Q);
                    tt[j] = t;
                    par ^= t;
                    const uint32_t key = ((uint32_t)(t < 0 ? -t : t) << 6) | (uint32_t)j;
                    min2 = min(min2, max(min1, key));
                    min1 = min(min1, key);
                }
            }
            if (FUSED) zodd |= hpar;
            const int idx = (int)(min1 & 63u);
            const int A = norm_q((int)(min1 >> 6), a8, bq);
            const int B = norm_q((int)(min2 >> 6), a8, bq);
            if (MSG == MSG_1BIT) cst[m] = (uint16_t)(A | (B << 5) | (idx << 10));
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < D) {
                    const int mag = (j == idx) ? B : A;
                    const bool neg = (par ^ tt[j]) < 0;
                    const int ln = neg ? -mag : mag;
                    if (MSG == MSG_INT8) {
                        L8[j * Mp + m] = (int8_t)ln;
                    } else {
                        const unsigned long long ball = __ballot(neg);
                        if ((m & 63) == 0) sgn[j * MpW + (m >> 6)] = ball;
                    }
                    const int delta = ln - lo[j];
                    if (delta != 0 && nid[j] != dummy) {
                        uint32_t w, sh;
                        zloc(nid[j], P, w, sh);
                        atomicAdd(&zacc[w], (uint32_t)delta << sh);
                    }
                }
            }
        }
        if (FUSED && k >= 2 && zodd < 0) flag[1 + (k & 1)] = 1;
        __syncthreads();
        if (FUSED && k >= 2 && flag[1 + (k & 1)] == 0) {  // Z^(k-1) is a codeword
            conv_prev = true;
            break;
        }
        // ---- variable pass: refresh the saturated gather copy
        if (tid == 0) *flag = 0;
        for (int w = tid; w < nwords; w += T) {
            const uint32_t v = zacc[w];
            for (int i = 0; i < P; ++i) {
                const int n = w * P + i;
                if (n < N) zold[n] = (ZT)clamp_i(zfield(v, (uint32_t)(i * zp.bits), zp), -Z2, Z2);
            }
        }
        __syncthreads();
        iters = k;
        if (!FUSED && a.early_stop) {
            syndrome_pass(tid, T, Mp, D, ell, zold, flag);
            __syncthreads();
            if (*flag == 0) {
                converged = true;
                break;
            }
        }
    }

    int ok = 1;
    if (!converged && !conv_prev) {
        __syncthreads();
        if (tid == 0) *flag = 0;
        __syncthreads();
        syndrome_pass(tid, T, Mp, D, ell, zold, flag);
        __syncthreads();
        ok = (*flag == 0);
    }
    // ---- outputs
    if (FUSED && conv_prev) {  // decisions of Z^(iters) from its saturated copy
        for (int n = tid; n < N; n += T) a.hard_out[(size_t)f * N + n] = zold[n] <= 0 ? 1 : 0;
    } else for (int n = tid; n < N; n += T) {
        uint32_t w, sh;
        zloc((uint32_t)n, P, w, sh);
        const int z = zfield(zacc[w], sh, zp);
        a.hard_out[(size_t)f * N + n] = z <= 0 ? 1 : 0;
        if (a.llr_out) a.llr_out[(size_t)f * N + n] = (float)((double)z * a.step);
    }
    if (tid == 0) {
        a.iters_out[f] = iters;
        a.ok_out[f] = (uint8_t)ok;
    }
}

template <int DMAX, int MSG, bool ML, bool FUSED, typename ZT>
hipError_t launch_one(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    auto kern = ss_int_kernel<DMAX, MSG, ML, FUSED, ZT>;
    if (c.lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_frames), dim3((unsigned)c.threads), c.lds, s, a);
    return hipGetLastError();
}

template <int DMAX, int MSG, typename ZT>
hipError_t launch_msg(const DecodeArgs &a, const LaunchCfg &c, hipStream_t s) {
    // the fused check needs at least one iteration and no posterior output
    if (a.early_stop && a.llr_out == nullptr && a.max_iter >= 1)
        return c.msg_lds ? launch_one<DMAX, MSG, true, true, ZT>(a, c, s)
                         : launch_one<DMAX, MSG, false, true, ZT>(a, c, s);
    return c.msg_lds ? launch_one<DMAX, MSG, true, false, ZT>(a, c, s)
                     : launch_one<DMAX, MSG, false, false, ZT>(a, c, s);
}

template <int DMAX>
hipError_t launch_dmax(const DecodeArgs &a, int msg, const LaunchCfg &c, hipStream_t s) {
    if (msg != MSG_INT8) return launch_msg<DMAX, MSG_1BIT, int8_t>(a, c, s);  // 1-bit state: 6-bit values
    return a.zmax > 127 ? launch_msg<DMAX, MSG_INT8, int16_t>(a, c, s) : launch_msg<DMAX, MSG_INT8, int8_t>(a, c, s);
}

}  // namespace

hipError_t launch_ss_int(const DecodeArgs &a, int msg, const LaunchCfg &c, hipStream_t s) {
    switch (c.dmax) {
        case 8: return launch_dmax<8>(a, msg, c, s);
        case 16: return launch_dmax<16>(a, msg, c, s);
        case 32: return launch_dmax<32>(a, msg, c, s);
        case 64: return launch_dmax<64>(a, msg, c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpc
