// Two-scan min-sum (Sec. III, Eqs. 1-2), the baseline schedule, with frames
// across lanes: one or four consecutive frames per lane (64 or 256 frames per
// wavefront), every per-frame array frame-minor (element (i, f) at i*Fp + f),
// so a wavefront's access to one value is one contiguous line and the code's
// addressing is wave-uniform.
//
// Both per-edge arrays of the schedule are kept in the caller's workspace,
// in the row order of H (CSR):
//   Z_mn  variable-to-check messages (Z^(0)_n initially)
//   L_mn  check-to-variable messages
// and each iteration is the paper's two scans:
//   horizontal (rows)     L_mn = prod sgn * norm(min |Z_mn'|) over n' != n,
//                         from min1/argmin/min2 and the sign parity of the row
//   vertical (variables)  Z_n = Z^(0)_n + sum of L_mn over M(n) (ascending
//                         check order), then every Z_mn as Eq. (2) writes it
//                         (fixed point: sat(Z_n - L_mn), the saturated
//                         exclusion sum exactly; binary32: its own sum
//                         Z^(0)_n + the other L_m'n in ascending check order)
// The vertical scan reaches the row-ordered arrays through the
// variable-to-check index: the second addressing table that the single-scan
// form does without.  Fixed point: 6-bit messages in int8, Z_n in int16.
// In binary32 the exclusion sums round differently from Z_n - L_mn (the
// single-scan extrinsic), so the two schedules are not bitwise equal there.
// Early stop and outputs as in the single-scan frames-across-lanes
// decoder (syndrome of Z^(k) formed in the horizontal scan of iteration k+1).
#include "fl_common.h"

#include <type_traits>

namespace ldpc {
namespace {

using namespace fl;

struct TsArgs {
    int32_t M, N, F, Fp, G;
    int32_t rwaves;
    uint32_t ebytes;   // bytes of each per-edge array
    uint32_t z0bytes;  // bytes of Z^(0)
    uint32_t znbytes;  // bytes of Z_n
    int32_t a8, b_int;
    float alpha, beta;
    const int32_t *row_ptr;   // [M+1]
    const uint32_t *row_ent;  // [E + 64][2] {variable, variable-major position} (padded)
    const int32_t *vc_ptr;    // [N+1]
    const uint32_t *vc_csr;   // [E + 64] row-order edge of each variable-major position (padded)
    void *z0;                 // [N][Fp] int8 / float
    void *zn;                 // [N][Fp] int16 / float
    void *zmn;                // [E][Fp] int8 / float, row order
    void *L;                  // [E][Fp] int8 / float, row order
    int32_t *fail;            // [K+1][Fp]
    int32_t *conv;            // [Fp]
};

// Z_n := Z^(0)_n (widened), the posterior before the first iteration.
template <class Tin, class Tz>
__global__ void __launch_bounds__(kBlock) widen_z0(const Tin *__restrict__ z0, Tz *__restrict__ zn, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) zn[i] = (Tz)z0[i];
}

__device__ __forceinline__ float norm_f(float m, float alpha, float beta) {
    const float v = __fsub_rn(__fmul_rn(alpha, m), beta);
    return v > 0.0f ? v : 0.0f;
}

__device__ __forceinline__ int norm_q(int m, int a8, int b) {
    const int v = ((m * a8 + 128) >> 8) - b;
    return v > 0 ? v : 0;
}

// V consecutive frames per lane (1 or 4) of one element in one access: int8
// messages (V bytes), int16 posteriors (2V bytes), binary32 (4V bytes).
template <int V>
__device__ __forceinline__ void ld_i8(const Buf &b, int (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (V == 4) {
        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(b.r, lo, eo, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = (int)(int8_t)(uint8_t)(x >> (8 * c));
    } else {
        v[0] = b.ld8(lo, eo);
    }
}
template <int V>
__device__ __forceinline__ void st_i8(const Buf &b, const int (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (V == 4) {
        const uint32_t x = ((uint32_t)v[0] & 255u) | (((uint32_t)v[1] & 255u) << 8) |
                           (((uint32_t)v[2] & 255u) << 16) | ((uint32_t)v[3] << 24);
        __builtin_amdgcn_raw_buffer_store_b32(x, b.r, lo, eo, 0);
    } else {
        b.st8(v[0], lo, eo);
    }
}
template <int V>
__device__ __forceinline__ void ld_i16(const Buf &b, int (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (V == 4) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(b.r, lo, eo, 0);
        const uint32_t w0 = x[0], w1 = x[1];
        v[0] = (int)(int16_t)(uint16_t)w0;
        v[1] = (int)(int16_t)(uint16_t)(w0 >> 16);
        v[2] = (int)(int16_t)(uint16_t)w1;
        v[3] = (int)(int16_t)(uint16_t)(w1 >> 16);
    } else {
        v[0] = b.ld16(lo, eo);
    }
}
template <int V>
__device__ __forceinline__ void st_i16(const Buf &b, const int (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (V == 4) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 x = {((uint32_t)v[0] & 0xFFFFu) | ((uint32_t)v[1] << 16),
                         ((uint32_t)v[2] & 0xFFFFu) | ((uint32_t)v[3] << 16)};
        __builtin_amdgcn_raw_buffer_store_b64(x, b.r, lo, eo, 0);
    } else {
        b.st16(v[0], lo, eo);
    }
}
// messages (int8 or binary32) and posteriors Z_n (int16 or binary32)
template <bool INT, int V, class T>
__device__ __forceinline__ void ld_msg(const Buf &b, T (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (INT)
        ld_i8<V>(b, v, lo, eo);
    else
        b.ldv<V, 0>(v, lo, eo);
}
template <bool INT, int V, class T>
__device__ __forceinline__ void st_msg(const Buf &b, const T (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (INT)
        st_i8<V>(b, v, lo, eo);
    else
        b.stv<V, 0>(v, lo, eo);
}
template <bool INT, int V, class T>
__device__ __forceinline__ void ld_post(const Buf &b, T (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (INT)
        ld_i16<V>(b, v, lo, eo);
    else
        b.ldv<V, 0>(v, lo, eo);
}
template <bool INT, int V, class T>
__device__ __forceinline__ void st_post(const Buf &b, const T (&v)[V], uint32_t lo, uint32_t eo) {
    if constexpr (INT)
        st_i16<V>(b, v, lo, eo);
    else
        b.stv<V, 0>(v, lo, eo);
}

// Horizontal scan of iteration k (UPDATE), or the syndrome of Z_n alone.
//   syn_row >= 0: rows failing the syndrome of Z_n set fail[syn_row]
//   conv_k  >= 1: first fold fail[conv_k] into conv (one wavefront)
// FIRST: Z_mn = Z^(0)_n, gathered from z0.  V frames per lane.
template <bool INT, int DMAX, bool UPDATE, bool FIRST, int V>
__global__ void __launch_bounds__(kBlock) ts_rows(TsArgs a, int syn_row, int conv_k) {
    constexpr uint32_t es = INT ? 1 : 4, zs = INT ? 2 : 4;
    using T = typename std::conditional<INT, int, float>::type;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (conv_k >= 1 && w == 0) fold_conv(a.conv, a.fail, conv_k, Fp, lane);
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * V);  // first frame of the lane
    const uint32_t foe = f0 * es, foz = f0 * zs;
    const uint32_t rowe = (uint32_t)Fp * es, rowz = (uint32_t)Fp * zs;
    const Buf b0(a.z0, a.z0bytes), bn(a.zn, a.znbytes), bm(a.zmn, a.ebytes), bl(a.L, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    const bool syn_on = syn_row >= 0;
    for (int m = w / a.G; m < a.M; m += a.rwaves) {
        const int e0 = rp[m];
        const int d = rp[m + 1] - e0;
        uint32_t vo0[DMAX], voz[DMAX], epos[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t nv = re[2 * (e0 + j)];
            vo0[j] = j < d ? nv * rowe : kOutOfRange;
            voz[j] = j < d ? nv * rowz : kOutOfRange;
            epos[j] = j < d ? (uint32_t)(e0 + j) * rowe : kOutOfRange;
        }
        // loads first (slots j >= d out of range), then the arithmetic
        T t[DMAX][V];
        T zv[DMAX][V];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (UPDATE) {
                if (FIRST)
                    ld_msg<INT, V>(b0, t[j], foe, vo0[j]);
                else
                    ld_msg<INT, V>(bm, t[j], foe, epos[j]);
            }
            if (syn_on) ld_post<INT, V>(bn, zv[j], foz, voz[j]);
        }
#pragma unroll
        for (int c = 0; c < V; ++c) {  // each frame on its own
            if (syn_on) {
                int syn = 0;
#pragma unroll
                for (int j = 0; j < DMAX; ++j) syn ^= (j < d && !(zv[j][c] > (T)0)) ? 1 : 0;
                if (syn) a.fail[(size_t)syn_row * Fp + f0 + c] = 1;
            }
            if (UPDATE) {
                int par = 0, idx = 0;
                T min1, min2;
                if constexpr (INT) {
                    min1 = 255;
                    min2 = 255;
                } else {
                    min1 = INFINITY;
                    min2 = INFINITY;
                }
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    const bool in = j < d;
                    par ^= (in && t[j][c] < (T)0) ? 1 : 0;
                    T av;
                    if constexpr (INT)
                        av = in ? abs(t[j][c]) : 255;
                    else
                        av = in ? fabsf(t[j][c]) : INFINITY;
                    if constexpr (INT) {
                        min2 = min(min2, max(min1, av));
                        idx = av < min1 ? j : idx;
                        min1 = min(min1, av);
                    } else {
                        min2 = fminf(min2, fmaxf(min1, av));
                        idx = av < min1 ? j : idx;
                        min1 = fminf(min1, av);
                    }
                }
                T A, B;
                if constexpr (INT) {
                    A = norm_q(min1, a.a8, a.b_int);
                    B = norm_q(min2, a.a8, a.b_int);
                } else {
                    A = norm_f(min1, a.alpha, a.beta);
                    B = norm_f(min2, a.alpha, a.beta);
                }
#pragma unroll
                for (int j = 0; j < DMAX; ++j) {
                    const T mag = j == idx ? B : A;
                    t[j][c] = (par ^ (t[j][c] < (T)0 ? 1 : 0)) ? -mag : mag;  // L_mn
                }
            }
        }
        if (UPDATE) {
#pragma unroll
            for (int j = 0; j < DMAX; ++j) st_msg<INT, V>(bl, t[j], foe, epos[j]);
        }
    }
}

// Vertical scan of iteration k: Z_n and the new Z_mn.  Frames frozen by the
// early stop keep their Z_n.  Variables of degree up to 8 keep their
// messages in registers between the sum and the extrinsics; larger degrees
// read them twice.  V frames per lane.
template <bool INT, bool FREEZE, int V>
__global__ void __launch_bounds__(kBlock) ts_vars(TsArgs a, int fail_row) {
    constexpr uint32_t es = INT ? 1 : 4, zs = INT ? 2 : 4;
    using T = typename std::conditional<INT, int, float>::type;
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * V);
    const uint32_t foe = f0 * es, foz = f0 * zs;
    const uint32_t rowe = (uint32_t)Fp * es, rowz = (uint32_t)Fp * zs;
    const Buf b0(a.z0, a.z0bytes), bn(a.zn, a.znbytes), bm(a.zmn, a.ebytes), bl(a.L, a.ebytes);
    bool frozen[V];
    bool any_frozen = false;
#pragma unroll
    for (int c = 0; c < V; ++c) {
        frozen[c] = FREEZE && (a.conv[f0 + c] != kNotConverged || a.fail[(size_t)fail_row * Fp + f0 + c] == 0);
        any_frozen = any_frozen || frozen[c];
    }
    // frozen frames keep Z_n: their old values are read back only by lanes
    // that hold one (an out-of-range offset moves no data)
    const uint32_t fc = (FREEZE && any_frozen) ? foz : kOutOfRange;
    const auto *vp = cptr(a.vc_ptr);
    const auto *vcs = cptr(a.vc_csr);
    auto st_ext = [&](const T (&zsum)[V], const T (&lv)[V], uint32_t off) {  // Z_mn = Z_n - L_mn
        T x[V];
#pragma unroll
        for (int c = 0; c < V; ++c) {
            if constexpr (INT) {
                const int v = zsum[c] - lv[c];
                x[c] = v > kQmax ? kQmax : (v < -kQmax ? -kQmax : v);
            } else {
                x[c] = __fsub_rn(zsum[c], lv[c]);
            }
        }
        st_msg<INT, V>(bm, x, foe, off);
    };
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const int e0 = vp[n], e1 = vp[n + 1];
        T s[V], cp[V], z0v[V];
        ld_msg<INT, V>(b0, s, foe, (uint32_t)n * rowe);
#pragma unroll
        for (int c = 0; c < V; ++c) z0v[c] = s[c];
        if (FREEZE) ld_post<INT, V>(bn, cp, fc, (uint32_t)n * rowz);
        T l[8][V];
        uint32_t eo[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) eo[i] = kOutOfRange;
        // Z_n: eight messages per step, all loads in flight together; slots
        // past the last edge are out of range and skipped (nothing is added)
        for (int e = e0; e < e1; e += 8) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t ce = vcs[e + i];
                eo[i] = e + i < e1 ? ce * rowe : kOutOfRange;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) ld_msg<INT, V>(bl, l[i], foe, eo[i]);
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    if constexpr (INT)
                        s[c] = e + i < e1 ? s[c] + l[i][c] : s[c];
                    else
                        s[c] = e + i < e1 ? __fadd_rn(s[c], l[i][c]) : s[c];
                }
        }
        {
            T zn[V];
#pragma unroll
            for (int c = 0; c < V; ++c) zn[c] = (FREEZE && frozen[c]) ? cp[c] : s[c];
            st_post<INT, V>(bn, zn, foz, (uint32_t)n * rowz);
        }
        // extrinsics: a variable of degree <= 8 still holds its messages and
        // their offsets in registers (out-of-range slots are dropped stores);
        // larger degrees read them again
        if constexpr (!INT) {
            // binary32, Eq. (2) as written: Z_mn = Z^(0)_n + the other L_m'n in
            // ascending check order.  x[i] starts from the prefix Z^(0) + l[0..i-1]
            // and adds l[i+1..]; degrees above 8 stream the other chunks again
            if (e1 - e0 <= 8) {
                const int deg = e1 - e0;
                T pre[V];
#pragma unroll
                for (int c = 0; c < V; ++c) pre[c] = z0v[c];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    T x[V];
#pragma unroll
                    for (int c = 0; c < V; ++c) x[c] = pre[c];
#pragma unroll
                    for (int j = i + 1; j < 8; ++j)
#pragma unroll
                        for (int c = 0; c < V; ++c) x[c] = j < deg ? __fadd_rn(x[c], l[j][c]) : x[c];
                    st_msg<INT, V>(bm, x, foe, eo[i]);
#pragma unroll
                    for (int c = 0; c < V; ++c) pre[c] = i < deg ? __fadd_rn(pre[c], l[i][c]) : pre[c];
                }
            } else {
                for (int e = e0; e < e1; e += 8) {  // eight outputs at a time
                    uint32_t oo[8];
                    T x[8][V];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        oo[i] = e + i < e1 ? vcs[e + i] * rowe : kOutOfRange;
#pragma unroll
                        for (int c = 0; c < V; ++c) x[i][c] = z0v[c];
                    }
                    for (int e2 = e0; e2 < e1; e2 += 8) {  // every input chunk, ascending
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const uint32_t ce = vcs[e2 + j];
                            eo[j] = e2 + j < e1 ? ce * rowe : kOutOfRange;
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j) ld_msg<INT, V>(bl, l[j], foe, eo[j]);
#pragma unroll
                        for (int i = 0; i < 8; ++i)
#pragma unroll
                            for (int j = 0; j < 8; ++j) {
                                const bool use = e2 + j < e1 && e2 + j != e + i;
#pragma unroll
                                for (int c = 0; c < V; ++c) x[i][c] = use ? __fadd_rn(x[i][c], l[j][c]) : x[i][c];
                            }
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) st_msg<INT, V>(bm, x[i], foe, oo[i]);
                }
            }
        } else if (e1 - e0 <= 8) {
#pragma unroll
            for (int i = 0; i < 8; ++i) st_ext(s, l[i], eo[i]);
        } else {
            for (int e = e0; e < e1; e += 8) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t ce = vcs[e + i];
                    eo[i] = e + i < e1 ? ce * rowe : kOutOfRange;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) ld_msg<INT, V>(bl, l[i], foe, eo[i]);
#pragma unroll
                for (int i = 0; i < 8; ++i) st_ext(s, l[i], eo[i]);
            }
        }
    }
}

// int8 with four frames per lane: two frames per 32-bit register in 16-bit
// halves (packed VALU), four int8 messages per 4-byte access, four int16
// posteriors per 8-byte access.  Same arithmetic as the kernels above.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ i16x2 as_i(uint32_t v) { return __builtin_bit_cast(i16x2, v); }
__device__ __forceinline__ uint32_t bits(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t bits(i16x2 v) { return __builtin_bit_cast(uint32_t, v); }
// four int8 of frames 0..3 -> (frames 0, 1) and (frames 2, 3), sign-extended
// 16-bit halves: each byte moved to the top of its half, then shifted back
__device__ __forceinline__ void unpack4(uint32_t x, uint32_t &p0, uint32_t &p1) {
    p0 = bits(as_i(__builtin_amdgcn_perm(x, x, 0x010c000cu)) >> (i16x2){8, 8});
    p1 = bits(as_i(__builtin_amdgcn_perm(x, x, 0x030c020cu)) >> (i16x2){8, 8});
}
// the low byte of each half of (frames 0, 1), (frames 2, 3) -> four int8
__device__ __forceinline__ uint32_t pack4(uint32_t p0, uint32_t p1) {
    return __builtin_amdgcn_perm(p1, p0, 0x06040200u);
}

template <int DMAX, bool UPDATE, bool FIRST>
__global__ void __launch_bounds__(kBlock) ts_rows_i8x4(TsArgs a, int syn_row, int conv_k) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (conv_k >= 1 && w == 0) fold_conv(a.conv, a.fail, conv_k, Fp, lane);
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * 4);  // first frame of the lane
    const uint32_t foe = f0, foz = f0 * 2u;
    const uint32_t rowe = (uint32_t)Fp, rowz = (uint32_t)Fp * 2u;
    const Buf b0(a.z0, a.z0bytes), bn(a.zn, a.znbytes), bm(a.zmn, a.ebytes), bl(a.L, a.ebytes);
    const auto *rp = cptr(a.row_ptr);
    const auto *re = cptr(a.row_ent);
    const bool syn_on = syn_row >= 0;
    // A, B = max(((m a8 + 128) >> 8) - b, 0) per half: m <= 127 keeps the
    // product below 2^15; offsets past 255 steps zero every magnitude anyway
    const u16x2 a8x2 = (u16x2){(unsigned short)a.a8, (unsigned short)a.a8};
    const short bq = (short)min(a.b_int, 255);
    const i16x2 bx2 = (i16x2){bq, bq};
    for (int m = w / a.G; m < a.M; m += a.rwaves) {
        const int e0 = rp[m];
        const int d = rp[m + 1] - e0;
        uint32_t vo0[DMAX], voz[DMAX], epos[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            const uint32_t nv = re[2 * (e0 + j)];
            vo0[j] = j < d ? nv * rowe : kOutOfRange;
            voz[j] = j < d ? nv * rowz : kOutOfRange;
            epos[j] = j < d ? (uint32_t)(e0 + j) * rowe : kOutOfRange;
        }
        uint32_t x[DMAX], za[DMAX], zb[DMAX];
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
            if (UPDATE)
                x[j] = FIRST ? __builtin_amdgcn_raw_buffer_load_b32(b0.r, foe, vo0[j], 0)
                             : __builtin_amdgcn_raw_buffer_load_b32(bm.r, foe, epos[j], 0);
            if (syn_on) {
                const auto zz = __builtin_amdgcn_raw_buffer_load_b64(bn.r, foz, voz[j], 0);
                za[j] = zz[0];
                zb[j] = zz[1];
            }
        }
        if (syn_on) {  // bits 15 / 31: odd number of Z_n <= 0 in the row (Z_n - 1 < 0)
            uint32_t h0 = 0, h1 = 0;
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                if (j < d) {
                    h0 ^= bits(as_i(za[j]) - (i16x2){1, 1});
                    h1 ^= bits(as_i(zb[j]) - (i16x2){1, 1});
                }
            }
            const uint32_t hb[4] = {h0 & 0x8000u, h0 & 0x80000000u, h1 & 0x8000u, h1 & 0x80000000u};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (hb[c]) a.fail[(size_t)syn_row * Fp + f0 + c] = 1;
        }
        if (UPDATE) {
            uint32_t t[2][DMAX], mg[2][DMAX];
            u16x2 mn1[2] = {{255, 255}, {255, 255}}, mn2[2] = {{255, 255}, {255, 255}};
            uint32_t par[2] = {0u, 0u};
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                unpack4(x[j], t[0][j], t[1][j]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // slots past the row's end read 0: no sign, magnitude forced to 255
                    par[h] ^= t[h][j];
                    const i16x2 tv = as_i(t[h][j]);
                    const u16x2 av = j < d ? as_u(bits(__builtin_elementwise_max(tv, -tv))) : (u16x2){255, 255};
                    mg[h][j] = bits(av);
                    mn2[h] = __builtin_elementwise_min(mn2[h], __builtin_elementwise_max(mn1[h], av));
                    mn1[h] = __builtin_elementwise_min(mn1[h], av);
                }
            }
            uint32_t A[2], B[2], ps[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                A[h] = bits(__builtin_elementwise_max(
                    as_i(bits((mn1[h] * a8x2 + (u16x2){128, 128}) >> (u16x2){8, 8})) - bx2, (i16x2){0, 0}));
                B[h] = bits(__builtin_elementwise_max(
                    as_i(bits((mn2[h] * a8x2 + (u16x2){128, 128}) >> (u16x2){8, 8})) - bx2, (i16x2){0, 0}));
                ps[h] = bits(as_i(par[h]) >> (i16x2){15, 15});
            }
#pragma unroll
            for (int j = 0; j < DMAX; ++j) {
                uint32_t L[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // |t_j| >= min1: (min1 - |t_j|) >> 15 is 0 at the minimum (B there,
                    // and at a tie, where B = A) and -1 elsewhere (A)
                    const uint32_t nsel =
                        bits(as_i(bits(mn1[h] - as_u(mg[h][j]))) >> (i16x2){15, 15});
                    const uint32_t mag = __builtin_amdgcn_bitop3_b32(nsel, A[h], B[h], 0xCA);  // nsel ? A : B
                    const uint32_t sg = __builtin_amdgcn_bitop3_b32(bits(as_i(t[h][j]) >> (i16x2){15, 15}), ps[h],
                                                                     0x00010001u, 0xBE);  // (a ^ b) | c
                    L[h] = bits(as_i(mag) * as_i(sg));
                }
                __builtin_amdgcn_raw_buffer_store_b32(pack4(L[0], L[1]), bl.r, foe, epos[j], 0);
            }
        }
    }
}

template <bool FREEZE>
__global__ void __launch_bounds__(kBlock) ts_vars_i8x4(TsArgs a, int fail_row) {
    const int lane = threadIdx.x & 63;
    const int w = wave_id();
    const int Fp = a.Fp;
    if (w >= a.rwaves * a.G) return;
    const int g = w % a.G;
    const uint32_t f0 = (uint32_t)((g * 64 + lane) * 4);
    const uint32_t foe = f0, foz = f0 * 2u;
    const uint32_t rowe = (uint32_t)Fp, rowz = (uint32_t)Fp * 2u;
    const Buf b0(a.z0, a.z0bytes), bn(a.zn, a.znbytes), bm(a.zmn, a.ebytes), bl(a.L, a.ebytes);
    // frozen frames keep Z_n: a mask per 16-bit half selects their old value
    uint32_t fm[2] = {0u, 0u};
    bool any_frozen = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool fz = FREEZE && (a.conv[f0 + c] != kNotConverged || a.fail[(size_t)fail_row * Fp + f0 + c] == 0);
        if (fz) fm[c >> 1] |= (c & 1) ? 0xFFFF0000u : 0x0000FFFFu;
        any_frozen = any_frozen || fz;
    }
    const uint32_t fc = (FREEZE && any_frozen) ? foz : kOutOfRange;
    const auto *vp = cptr(a.vc_ptr);
    const auto *vcs = cptr(a.vc_csr);
    // Z_mn = sat(Z_n - L_mn) to +-Q for both pairs, stored as four int8
    auto st_ext = [&](const uint32_t (&sz)[2], const uint32_t (&lv)[2], uint32_t off) {
        uint32_t e[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            e[h] = bits(__builtin_elementwise_min(
                __builtin_elementwise_max(as_i(sz[h]) - as_i(lv[h]), (i16x2){-kQmax, -kQmax}), (i16x2){kQmax, kQmax}));
        __builtin_amdgcn_raw_buffer_store_b32(pack4(e[0], e[1]), bm.r, foe, off, 0);
    };
    for (int n = w / a.G; n < a.N; n += a.rwaves) {
        const int e0 = vp[n], e1 = vp[n + 1];
        uint32_t sz[2], cp[2] = {0u, 0u};
        unpack4(__builtin_amdgcn_raw_buffer_load_b32(b0.r, foe, (uint32_t)n * rowe, 0), sz[0], sz[1]);
        if (FREEZE) {
            const auto c2 = __builtin_amdgcn_raw_buffer_load_b64(bn.r, fc, (uint32_t)n * rowz, 0);
            cp[0] = c2[0];
            cp[1] = c2[1];
        }
        uint32_t l[8][2];
        uint32_t eo[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) eo[i] = kOutOfRange;
        // Z_n: eight messages per step, all loads in flight together; slots
        // past the last edge are out of range and skipped (nothing is added)
        for (int e = e0; e < e1; e += 8) {
            uint32_t raw[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t ce = vcs[e + i];
                eo[i] = e + i < e1 ? ce * rowe : kOutOfRange;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) raw[i] = __builtin_amdgcn_raw_buffer_load_b32(bl.r, foe, eo[i], 0);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                unpack4(raw[i], l[i][0], l[i][1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) sz[h] = e + i < e1 ? bits(as_i(sz[h]) + as_i(l[i][h])) : sz[h];
            }
        }
        {
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            const u32x2 zn = {(uint32_t)__builtin_amdgcn_bitop3_b32(fm[0], cp[0], sz[0], 0xCA),  // frozen ? old : new
                              (uint32_t)__builtin_amdgcn_bitop3_b32(fm[1], cp[1], sz[1], 0xCA)};
            __builtin_amdgcn_raw_buffer_store_b64(zn, bn.r, foz, (uint32_t)n * rowz, 0);
        }
        // extrinsics: a variable of degree <= 8 still holds its messages and
        // their offsets in registers (out-of-range slots are dropped stores);
        // larger degrees read them again
        if (e1 - e0 <= 8) {
#pragma unroll
            for (int i = 0; i < 8; ++i) st_ext(sz, l[i], eo[i]);
        } else {
            for (int e = e0; e < e1; e += 8) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t ce = vcs[e + i];
                    eo[i] = e + i < e1 ? ce * rowe : kOutOfRange;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    unpack4(__builtin_amdgcn_raw_buffer_load_b32(bl.r, foe, eo[i], 0), l[i][0], l[i][1]);
#pragma unroll
                for (int i = 0; i < 8; ++i) st_ext(sz, l[i], eo[i]);
            }
        }
    }
}

template <bool INT, int DMAX, int V>
hipError_t run(const DecodeArgs &d, const TsArgs &a, int K, unsigned grid, hipStream_t s) {
    using Tin = typename std::conditional<INT, int8_t, float>::type;
    using Tz = typename std::conditional<INT, int16_t, float>::type;
    const bool es = d.early_stop != 0;
    const dim3 tgrid((unsigned)((a.N + 63) / 64), (unsigned)(a.Fp / 64));
    hipLaunchKernelGGL(transpose_in<Tin>, tgrid, dim3(kBlock), 0, s, static_cast<const Tin *>(d.llr_in),
                       static_cast<Tin *>(a.z0), a.N, a.F, a.Fp);
    const int64_t nfail = (int64_t)(K + 1) * a.Fp;
    hipLaunchKernelGGL(init_flags, dim3((unsigned)((std::max<int64_t>(nfail, a.Fp) + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, a.fail, nfail, a.conv, a.Fp);
    // Z_n starts as Z^(0): the syndrome and the outputs of max_iter = 0
    const int64_t nz = (int64_t)a.N * a.Fp;
    hipLaunchKernelGGL((widen_z0<Tin, Tz>), dim3((unsigned)std::min<int64_t>((nz + kBlock - 1) / kBlock, 65536)),
                       dim3(kBlock), 0, s, static_cast<const Tin *>(a.z0), static_cast<Tz *>(a.zn), nz);
    constexpr bool kPacked = INT && V == 4;  // two frames per register
    for (int k = 1; k <= K; ++k) {
        const int syn_row = (es && k >= 2) ? k - 1 : -1;
        const int conv_k = (es && k >= 3) ? k - 2 : 0;
        if constexpr (kPacked) {
            if (k == 1)
                hipLaunchKernelGGL((ts_rows_i8x4<DMAX, true, true>), dim3(grid), dim3(kBlock), 0, s, a, syn_row,
                                   conv_k);
            else
                hipLaunchKernelGGL((ts_rows_i8x4<DMAX, true, false>), dim3(grid), dim3(kBlock), 0, s, a, syn_row,
                                   conv_k);
            if (es && k >= 2)
                hipLaunchKernelGGL((ts_vars_i8x4<true>), dim3(grid), dim3(kBlock), 0, s, a, k - 1);
            else
                hipLaunchKernelGGL((ts_vars_i8x4<false>), dim3(grid), dim3(kBlock), 0, s, a, 0);
        } else {
            if (k == 1)
                hipLaunchKernelGGL((ts_rows<INT, DMAX, true, true, V>), dim3(grid), dim3(kBlock), 0, s, a, syn_row,
                                   conv_k);
            else
                hipLaunchKernelGGL((ts_rows<INT, DMAX, true, false, V>), dim3(grid), dim3(kBlock), 0, s, a, syn_row,
                                   conv_k);
            if (es && k >= 2)
                hipLaunchKernelGGL((ts_vars<INT, true, V>), dim3(grid), dim3(kBlock), 0, s, a, k - 1);
            else
                hipLaunchKernelGGL((ts_vars<INT, false, V>), dim3(grid), dim3(kBlock), 0, s, a, 0);
        }
    }
    if constexpr (kPacked)
        hipLaunchKernelGGL((ts_rows_i8x4<DMAX, false, false>), dim3(grid), dim3(kBlock), 0, s, a, K,
                           (es && K >= 3) ? K - 2 : 0);
    else
        hipLaunchKernelGGL((ts_rows<INT, DMAX, false, false, V>), dim3(grid), dim3(kBlock), 0, s, a, K,
                           (es && K >= 3) ? K - 2 : 0);
    hipLaunchKernelGGL(frame_out, dim3((unsigned)((a.F + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a.fail, a.conv,
                       a.F, a.Fp, K, d.early_stop, d.iters_out, d.ok_out);
    hipLaunchKernelGGL(transpose_out<Tz>, tgrid, dim3(kBlock), 0, s, static_cast<const Tz *>(a.zn), a.N, a.F, a.Fp,
                       d.step, d.hard_out, d.llr_out);
    return hipGetLastError();
}

template <bool INT, int V>
hipError_t run_deg(const DecodeArgs &d, const TsArgs &a, int K, unsigned grid, hipStream_t s, int max_row_deg) {
    if (max_row_deg <= 8) return run<INT, 8, V>(d, a, K, grid, s);
    if (max_row_deg <= 16) return run<INT, 16, V>(d, a, K, grid, s);
    if constexpr (V == 1) {
        if (max_row_deg <= 32) return run<INT, 32, 1>(d, a, K, grid, s);
        return run<INT, 64, 1>(d, a, K, grid, s);
    }
    return hipErrorInvalidValue;  // four frames per lane take rows of at most 16 entries
}

// Chunk of a call (frames) and frames per lane of its plan: four per lane
// (one 4-, 8- or 16-byte access per element) once a chunk holds 256 frames,
// chunks then a multiple of 256.
struct TsPlan {
    int V, chunk;
};
TsPlan ts_plan(int N, int64_t E, bool int8, int n_frames) {
    const int chunk = ts_fl_chunk_frames(N, E, int8);
    if (std::min(n_frames, chunk) >= 256) return {4, chunk / 256 * 256};
    return {1, chunk};
}
size_t ts_round_frames(int F, int V) { return (size_t)((F + 64 * V - 1) / (64 * V)) * 64 * V; }

}  // namespace

int ts_fl_chunk_frames(int N, int64_t E, bool int8) {
    return fl::chunk_frames(std::max<int64_t>(E * (int8 ? 1 : 4), (int64_t)N * 4));
}

// Rows above 16 entries keep one frame per lane (four frames of a wide row
// would take the registers that hide the gathers' latency); the frame padding
// of the plan stays.
int ts_fl_frames_per_lane(int N, int64_t E, bool int8, int n_frames, int max_row_deg) {
    return (ts_plan(N, E, int8, n_frames).V == 4 && max_row_deg <= 16) ? 4 : 1;
}

size_t ts_fl_workspace_bytes(int N, int64_t E, int n_frames, int max_iter, bool int8) {
    const TsPlan pl = ts_plan(N, E, int8, n_frames);
    const int fr = std::min(n_frames, std::max(pl.chunk, 1));
    const size_t Fp = ts_round_frames(fr, pl.V);
    const size_t es = int8 ? 1 : 4, zs = int8 ? 2 : 4;
    return fl::al256((size_t)N * Fp * es) + fl::al256((size_t)N * Fp * zs) + 2 * fl::al256((size_t)E * Fp * es) +
           fl::al256((size_t)(max_iter + 1) * Fp * 4) + fl::al256(Fp * 4);
}

hipError_t launch_two_scan_fl(const DecodeArgs &d, bool int8, const int32_t *row_ptr, const uint32_t *row_ent,
                              const uint32_t *vc_csr, int64_t E, int max_row_deg, int cu_count, hipStream_t s) {
    const TsPlan pl = ts_plan(d.c.N, E, int8, d.n_frames);
    const int chunk = pl.chunk;
    if (chunk <= 0 || max_row_deg > 64) return hipErrorInvalidValue;
    const int V = ts_fl_frames_per_lane(d.c.N, E, int8, d.n_frames, max_row_deg);
    const size_t es = int8 ? 1 : 4, zs = int8 ? 2 : 4;
    for (int c0 = 0; c0 < d.n_frames; c0 += chunk) {
        const int F = std::min(chunk, d.n_frames - c0);
        DecodeArgs dc = d;
        dc.n_frames = F;
        dc.llr_in = static_cast<const uint8_t *>(d.llr_in) + (size_t)c0 * d.c.N * es;
        dc.hard_out = d.hard_out + (size_t)c0 * d.c.N;
        dc.llr_out = d.llr_out ? d.llr_out + (size_t)c0 * d.c.N : nullptr;
        dc.iters_out = d.iters_out + c0;
        dc.ok_out = d.ok_out + c0;
        TsArgs a{};
        a.M = d.c.M;
        a.N = d.c.N;
        a.F = F;
        a.Fp = (int)ts_round_frames(F, pl.V);
        a.G = a.Fp / (64 * V);
        a.a8 = d.a8;
        a.b_int = d.b_int;
        a.alpha = d.alpha;
        a.beta = d.beta;
        a.row_ptr = row_ptr;
        a.row_ent = row_ent;
        a.vc_ptr = d.c.vc_ptr;
        a.vc_csr = vc_csr;
        const size_t Fp = (size_t)a.Fp;
        a.ebytes = (uint32_t)((size_t)E * Fp * es);
        a.z0bytes = (uint32_t)((size_t)a.N * Fp * es);
        a.znbytes = (uint32_t)((size_t)a.N * Fp * zs);
        uint8_t *p = d.ws;
        a.z0 = p;
        p += fl::al256(a.z0bytes);
        a.zn = p;
        p += fl::al256(a.znbytes);
        a.zmn = p;
        p += fl::al256(a.ebytes);
        a.L = p;
        p += fl::al256(a.ebytes);
        a.fail = reinterpret_cast<int32_t *>(p);
        p += fl::al256((size_t)(d.max_iter + 1) * Fp * 4);
        a.conv = reinterpret_cast<int32_t *>(p);
        unsigned grid;
        wave_layout(cu_count, a.G, std::max(a.M, a.N), &a.rwaves, &grid);
        const int K = d.max_iter;
        hipError_t e;
        if (int8)
            e = V == 4 ? run_deg<true, 4>(dc, a, K, grid, s, max_row_deg)
                       : run_deg<true, 1>(dc, a, K, grid, s, max_row_deg);
        else
            e = V == 4 ? run_deg<false, 4>(dc, a, K, grid, s, max_row_deg)
                       : run_deg<false, 1>(dc, a, K, grid, s, max_row_deg);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ldpc
