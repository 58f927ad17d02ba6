// Register-resident single-scan min-sum in 6-bit fixed point (Sec. IV, Eq. 3;
// Sec. V for the 1-bit form).  One 1024-thread workgroup per frame; thread t
// owns the check rows m = k*1024 + t (k < R) for the whole decode and keeps
// their messages in VGPRs:
//   INT8  D int8 messages per row, four to a register;
//   1BIT  one register per row: D sign bits, then A, B (5 bits each) and the
//         argmin position n~ (5 bits): the compressed state of Sec. V (rows of
//         more than 17 slots: the signs in one register, A | B | n~ in another).
// The only per-edge memory traffic is the shared check-to-variable index
// (buffer loads from L2) plus two LDS operations: the gather of the saturated
// posterior and, when the message changed, the atomic add of L_new - L_old
// into the packed posterior accumulator.  Same arithmetic as ss_int.hip:
//   t = Z_old[n] - L_old with |t| saturated to 31 once per row, after the
//   row minimum (saturating before or after selects the same messages),
//   min1/argmin/min2 keyed as |t| << 5 | j.  Padding slots point at a
//   variable whose accumulator word holds nothing else, so their updates
//   need no test.
// Early stop with hard decisions only (FUSED) forms the syndrome of the
// hard decisions of Z^(k-1) from the Z_old gathers of iteration k, as in
// ss_pk.hip; with posterior output a separate check pass follows each
// iteration.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr int kT = kRegThreads;  // workgroup size of this family
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, gfx9 family

template <int P>
struct ZP;
template <>
struct ZP<1> {
    static constexpr int bits = 32;
    static constexpr int bias = 0;
    __device__ static void loc(uint32_t n, uint32_t &addr, uint32_t &sh) {
        addr = n << 2;
        sh = 0;
    }
};
template <>
struct ZP<2> {
    static constexpr int bits = 16;
    static constexpr int bias = 1 << 15;
    __device__ static void loc(uint32_t n, uint32_t &addr, uint32_t &sh) {
        addr = (n >> 1) << 2;
        sh = (n & 1u) << 4;
    }
};
template <>
struct ZP<3> {
    static constexpr int bits = 10;
    static constexpr int bias = 1 << 9;
    // n / 3 via a 24-bit multiply: exact for n < 98303 (the planner checks).
    // __umul24 returns a signed int; the product exceeds 2^31 for n >= 49152,
    // so it must be shifted as unsigned.
    __device__ static void loc(uint32_t n, uint32_t &addr, uint32_t &sh) {
        const uint32_t w = (uint32_t)__umul24(n, 43691u) >> 17;
        addr = w << 2;
        sh = (uint32_t)__umul24(n - 3u * w, 10u);
    }
};

template <int P>
__device__ __forceinline__ int zfield(uint32_t v, int i) {
    if (P == 1) return (int)v;
    return (int)((v >> (i * ZP<P>::bits)) & ((1u << ZP<P>::bits) - 1u)) - ZP<P>::bias;
}

__device__ __forceinline__ int norm_q(uint32_t mag, uint32_t a8, int b) {
    mag = min(mag, (uint32_t)kQmax);
    const int v = (int)(((uint32_t)__umul24(mag, a8) + 128u) >> 8) - b;
    return v > 0 ? v : 0;
}

// Pack the low bytes of four values into one register (v_perm_b32).
__device__ __forceinline__ uint32_t pack4(int b0, int b1, int b2, int b3) {
    const uint32_t lo = __builtin_amdgcn_perm((uint32_t)b1, (uint32_t)b0, 0x0c0c0400u);
    const uint32_t hi = __builtin_amdgcn_perm((uint32_t)b3, (uint32_t)b2, 0x0c0c0400u);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

__device__ __forceinline__ uint32_t ld_idx(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

template <int D, int R, int P, int MSG, bool FUSED>
__global__ void __launch_bounds__(kT) ss_reg_kernel(DecodeArgs a) {
    static_assert(D >= 2 && D <= 32, "slots per row");
    constexpr bool kWide1 = MSG == MSG_1BIT && D + 15 > 32;  // 1-bit state in two registers
    constexpr int W = MSG == MSG_INT8 ? (D + 3) / 4 : (kWide1 ? 2 : 1);
    constexpr int Mr = R * kT;
    extern __shared__ __align__(16) uint8_t lds[];
    const int tid = threadIdx.x;
    const int f = blockIdx.x;
    const int N = a.c.N;
    const uint32_t dummy = (uint32_t)a.c.dummy;
    int8_t *zold = reinterpret_cast<int8_t *>(lds + a.off_zold);  // Z_old saturated to +-62
    uint8_t *zacc_b = lds + a.off_zacc;
    uint32_t *zacc = reinterpret_cast<uint32_t *>(zacc_b);
    int *flag = reinterpret_cast<int *>(lds + a.off_aux);  // [0]: separate check, [1], [2]: fused
    const int8_t *__restrict__ z0 = static_cast<const int8_t *>(a.llr_in) + (size_t)f * N;
    const __amdgpu_buffer_rsrc_t ellr =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.c.ell_reg, (short)0, D * Mr * 4, kRsrcWord3);
    const int nwords = (int)(dummy / P) + 1;

    // ---- initialisation
    for (int w = tid; w < nwords; w += kT) {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int n = w * P + i;
            const int z = n < N ? min(max((int)z0[n], -kQmax), kQmax) : 0;
            v |= (uint32_t)(z + ZP<P>::bias) << (i * ZP<P>::bits);
        }
        zacc[w] = v;
    }
    for (int n = tid; n <= (int)dummy; n += kT)
        zold[n] = (int8_t)(n < N ? min(max((int)z0[n], -kQmax), kQmax) : (n == (int)dummy ? kZoldMax : 0));
    if (tid == 0) {
        flag[0] = 0;
        flag[1] = 0;
        flag[2] = 0;
    }

    uint32_t Lw[R][W];  // INT8: int8 messages; 1BIT: Lw[k][0] = state word
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int i = 0; i < W; ++i) Lw[k][i] = 0u;
    __syncthreads();

    const uint32_t tid4 = (uint32_t)tid * 4u;
    uint32_t a8 = (uint32_t)a.a8;  // normalisation pair
    int bq = a.b_int;
    int iters = 0;
    bool converged = false;  // the decision of the last completed iteration is a codeword
    bool conv_prev = false;  // FUSED: that of the iteration before the last one is
    for (int it = 1; it <= a.max_iter; ++it) {
        // FUSED: the sign bit collects odd hard-decision parities of Z^(it-1)
        // rows; flag[1 + (it & 1)] is set by this iteration and read after its
        // first barrier, the other one (read last iteration) is cleared here
        int zodd = 0;
        if (FUSED && tid == 0) flag[1 + ((it + 1) & 1)] = 0;
        if (a.wsched) {  // per-iteration pair (Sec. III's lambda_k, beta_k)
            int a8i;
            sched_pair(a, it, a8i, bq);
            a8 = (uint32_t)a8i;
        }
        // indices of the next row are loaded one row ahead; the scheduling
        // barriers keep the unrolled rows from hoisting every load to the top
        // The index stream is the same every iteration; an opaque zero added to
        // the scalar offset stops the compiler from hoisting all R*D loads out
        // of the iteration loop and pinning every index in a VGPR.
        uint32_t it0 = 0;
        asm volatile("" : "+s"(it0));
        // With few rows per thread the next row's indices are loaded one row
        // ahead; with many, registers are too scarce and other waves hide the
        // L2 latency instead.
        constexpr bool kPrefetch = R <= 16;
        uint32_t nn[D];
#pragma unroll
        for (int j = 0; j < D; ++j) nn[j] = kPrefetch ? ld_idx(ellr, tid4, it0 + (uint32_t)(j * Mr * 4)) : 0u;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t n[D];
            int traw[D];
            int lo[D];  // L_old
#pragma unroll
            for (int j = 0; j < D; ++j)  // row offset in the scalar operand: one address VGPR
                n[j] = kPrefetch ? nn[j] : ld_idx(ellr, tid4, it0 + (uint32_t)((j * Mr + k * kT) * 4));
            if (kPrefetch && k + 1 < R) {
#pragma unroll
                for (int j = 0; j < D; ++j) nn[j] = ld_idx(ellr, tid4, it0 + (uint32_t)((j * Mr + (k + 1) * kT) * 4));
            }
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (MSG == MSG_INT8) {
#pragma unroll
                for (int j = 0; j < D; ++j) lo[j] = (int)(int8_t)(Lw[k][j >> 2] >> (8 * (j & 3)));
            } else {
                const uint32_t s = Lw[k][0];
                uint32_t fs;  // A | B << 5 | n~ << 10
                if constexpr (kWide1)
                    fs = Lw[k][1];
                else
                    fs = s >> D;
                const int Ao = (int)(fs & 31u), Bo = (int)((fs >> 5) & 31u);
                const int Io = (int)((fs >> 10) & 31u);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int fv = (j == Io) ? Bo : Ao;
                    lo[j] = ((s >> j) & 1u) ? -fv : fv;
                }
            }
            uint32_t min1 = 0xFFFFFFFFu, min2 = 0xFFFFFFFFu;
            int par = 0, hpar = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int zv = (int)zold[n[j]];
                const int tr = zv - lo[j];  // Z_old - L_old
                traw[j] = tr;
                par ^= tr;
                if (FUSED) hpar ^= zv - 1;  // sign bit: Z_old <= 0
                const uint32_t key = ((uint32_t)(tr < 0 ? -tr : tr) << 5) | (uint32_t)j;
                min2 = min(min2, max(min1, key));
                min1 = min(min1, key);
            }
            if (FUSED) {  // opaque: otherwise the XOR chain is deferred and every gathered value stays live
                asm volatile("" : "+v"(hpar));
                zodd |= hpar;
            }
            const int idx = (int)(min1 & 31u);
            int A = norm_q(min1 >> 5, a8, bq);
            int B = norm_q(min2 >> 5, a8, bq);
            // computed once per row: keep the compiler from re-deriving them per edge
            asm volatile("" : "+v"(A), "+v"(B));
            int ln[D];
            uint32_t sbits = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int mag = (j == idx) ? B : A;
                const int sm = (par ^ traw[j]) >> 31;  // 0 or -1: sign of the other inputs' product
                ln[j] = (mag ^ sm) - sm;
                if (MSG == MSG_1BIT) sbits |= (uint32_t)(sm & 1) << j;
                const int delta = ln[j] - lo[j];
                if (delta != 0) {
                    uint32_t addr, sh;
                    ZP<P>::loc(n[j], addr, sh);
                    atomicAdd(reinterpret_cast<uint32_t *>(zacc_b + addr), (uint32_t)delta << sh);
                }
            }
            if constexpr (MSG == MSG_INT8) {
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const int j = 4 * i;
                    Lw[k][i] = pack4(ln[j], j + 1 < D ? ln[j + 1] : 0, j + 2 < D ? ln[j + 2] : 0,
                                     j + 3 < D ? ln[j + 3] : 0);
                }
            } else if constexpr (kWide1) {
                Lw[k][0] = sbits;
                Lw[k][1] = (uint32_t)A | ((uint32_t)B << 5) | ((uint32_t)idx << 10);
            } else {
                Lw[k][0] = sbits | ((uint32_t)A << D) | ((uint32_t)B << (D + 5)) | ((uint32_t)idx << (D + 10));
            }
            // Opaque at the loop back-edge: otherwise the compiler carries the
            // unpacked fields (A, B, n~, each message) into the next iteration
            // instead of the packed words, multiplying the live registers.
#pragma unroll
            for (int i = 0; i < W; ++i) asm volatile("" : "+v"(Lw[k][i]));
            __builtin_amdgcn_sched_barrier(0);
        }
        if (FUSED && it >= 2 && zodd < 0) flag[1 + (it & 1)] = 1;
        __syncthreads();
        if (FUSED && it >= 2 && flag[1 + (it & 1)] == 0) {  // Z^(it-1) is a codeword
            conv_prev = true;
            break;
        }
        if (tid == 0) *flag = 0;
        for (int w = tid; w < nwords; w += kT) {
            const uint32_t v = zacc[w];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int n = w * P + i;
                if (n < N) zold[n] = (int8_t)min(max(zfield<P>(v, i), -kZoldMax), kZoldMax);
            }
        }
        __syncthreads();
        iters = it;
        if (!FUSED && a.early_stop) {
            for (int k = 0; k < R; ++k) {
                const uint32_t voff = (uint32_t)(k * kT + tid) * 4u;
                int p = 0;
                for (int j = 0; j < D; ++j) p ^= (zold[ld_idx(ellr, voff, (uint32_t)(j * Mr * 4))] <= 0) ? 1 : 0;
                if (p) atomicOr(flag, 1);
            }
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
        for (int k = 0; k < R; ++k) {
            const uint32_t voff = (uint32_t)(k * kT + tid) * 4u;
            int p = 0;
            for (int j = 0; j < D; ++j) p ^= (zold[ld_idx(ellr, voff, (uint32_t)(j * Mr * 4))] <= 0) ? 1 : 0;
            if (p) atomicOr(flag, 1);
        }
        __syncthreads();
        ok = (*flag == 0);
    }
    if (FUSED && conv_prev) {  // decisions of Z^(iters) from its saturated copy
        for (int n = tid; n < N; n += kT) a.hard_out[(size_t)f * N + n] = zold[n] <= 0 ? 1 : 0;
    } else for (int n = tid; n < N; n += kT) {
        uint32_t addr, sh;
        ZP<P>::loc((uint32_t)n, addr, sh);
        const uint32_t v = *reinterpret_cast<const uint32_t *>(zacc_b + addr);
        const int z = (P == 1) ? (int)v : (int)((v >> sh) & ((1u << ZP<P>::bits) - 1u)) - ZP<P>::bias;
        a.hard_out[(size_t)f * N + n] = z <= 0 ? 1 : 0;
        if (a.llr_out) a.llr_out[(size_t)f * N + n] = (float)((double)z * a.step);
    }
    if (tid == 0) {
        a.iters_out[f] = iters;
        a.ok_out[f] = (uint8_t)ok;
    }
}

template <int D, int R, int P, int MSG, bool FUSED>
hipError_t launch_one(const DecodeArgs &a, size_t lds, hipStream_t s) {
    auto kern = ss_reg_kernel<D, R, P, MSG, FUSED>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_frames), dim3(kT), lds, s, a);
    return hipGetLastError();
}

template <int D, int R, int P, int MSG>
hipError_t launch_es(const DecodeArgs &a, size_t lds, hipStream_t s) {
    // the fused check needs at least one iteration and no posterior output
    if (a.early_stop && a.llr_out == nullptr && a.max_iter >= 1) return launch_one<D, R, P, MSG, true>(a, lds, s);
    return launch_one<D, R, P, MSG, false>(a, lds, s);
}

}  // namespace

// Instantiated (slots per row, rows per thread, accumulator packing) shapes.
// The planner picks the smallest shape that covers the code; anything else
// runs on the generic kernels.
#define LDPC_REG_SHAPES(X) \
    X(6, 1, 1)             \
    X(6, 2, 1)             \
    X(6, 4, 1)             \
    X(7, 8, 1)             \
    X(7, 16, 1)            \
    X(7, 16, 2)            \
    X(7, 32, 3)            \
    X(8, 8, 1)             \
    X(8, 16, 2)            \
    X(8, 32, 3)            \
    X(21, 3, 1)            \
    X(24, 2, 1)            \
    X(24, 4, 1)

bool reg_shape_available(int D, int R, int P) {
#define X(d, r, p) \
    if (D == d && R == r && P == p) return true;
    LDPC_REG_SHAPES(X)
#undef X
    return false;
}

void reg_shapes(int *out, int cap, int *count) {
    int i = 0;
#define X(d, r, p)               \
    if (i < cap) {               \
        out[3 * i] = d;          \
        out[3 * i + 1] = r;      \
        out[3 * i + 2] = p;      \
    }                            \
    ++i;
    LDPC_REG_SHAPES(X)
#undef X
    *count = i;
}

hipError_t launch_ss_reg(const DecodeArgs &a, int msg, int D, int R, int P, size_t lds, hipStream_t s) {
#define X(d, r, p)                                                                         \
    if (D == d && R == r && P == p) {                                                      \
        if (msg == MSG_INT8) return launch_es<d, r, p, MSG_INT8>(a, lds, s);               \
        return launch_es<d, r, p, MSG_1BIT>(a, lds, s);                                    \
    }
    LDPC_REG_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace ldpc
