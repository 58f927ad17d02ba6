// Register-resident single-scan min-sum, int8 messages or the 1-bit state of
// Sec. V, two check rows per thread processed together in the low and high
// halves of 32-bit registers (packed 16-bit VALU).  Same method and results
// as ss_reg.hip (Sec. IV, Eq. 3, 6-bit fixed point); only the instruction
// mapping differs:
//
//   thread t of T owns the rows a = p*T + t and b = (p + R/2)*T + t for
//   p < R/2; for every slot j the pair (row a, row b) is one 16-bit lane pair:
//     t2   = Zold2 - Lold2                  (both stored +63: v_pk_add_f16
//            on the stored integers read as binary16 subnormals, which is
//            exact and gives sign and magnitude; v_pk_sub_i16 for the
//            16-bit Z_old of 8-bit messages)
//     m2   = |t2|                           (one mask of the sign bits)
//     min2 = min(min2, max(min1, m2)), min1 = min(min1, m2)   (v_pk_*_u16)
//     parity ^= t2                          (sign bits 15 and 31)
//   per pair of rows: A2, B2 = normalised min1/min2;
//     mag2 = max(A2, B2 + 64 min1 - 64 |t2|)   (one multiply-add, one max;
//            int8 messages of 6-7 bits), or a bit-select of A2 / B2 on the
//            mask (min1 - |t2|) >> 15 (the 1-bit state, 8-bit messages)
//   i.e. B where |t_j| equals the row minimum and A elsewhere: no argmin is
//   needed, since a tie at the minimum forces min2 = min1 and so A = B.
//     L2   = mag2 * (+-1: own sign XOR row parity) + 63, delta2 = L2 - Lold2
//            (6-7 bit int8 messages: a binary16 multiply-add on subnormals)
//   and one LDS atomic per edge adds the delta into the posterior field.
// The binary16 forms rely on subnormals being kept, the default binary16
// denormal mode of a kernel (the build passes no fast-math flag); the
// bit-exact parity tests would fail at once if they were flushed.
//
// Variables live in LDS "slots" chosen at code creation: slot s holds Z_old
// in byte s and the accumulator in field s%P of word s/P, and the placement
// spreads the variables each half-wavefront touches over the LDS banks.  The
// slot table maps variables to slots only at load and store time.
//
// Per-slot index record (host-built, 16 bytes, coalesced per wavefront):
//   { s_a, s_b, acc_a, acc_b },  acc = LDS byte address of the accumulator
//   word; and per row pair the field shifts of its accumulator words, one
//   byte per edge (16 bytes per eight slots: one more load per row pair).
// The byte address and shift encode any accumulator packing, so the kernel
// needs no division by the field count; bytes 0, 2 and 3 of a shift word feed
// the shifts of the deltas as operands with no extraction (byte 1 after one
// shift right).  Against a combined record word ((address << 5) | shift),
// which needs a shift right per atomic address, this removes two VALU
// instructions per slot and row pair for one texture-addresser load per row
// pair (measured faster on every workload shape).  Padding entries of short
// rows read the dummy slot (Z_old at its maximum, never the row minimum) and
// add into a private word per lane.
// Z_old is stored as Z + 63 (bytes), messages as L + 63: a stored Z_old byte
// has bit 6 clear exactly when Z_old <= 0.
//
// Early stop (FUSED, for callers that want hard decisions only): the gather
// of iteration k already reads every Z^(k-1) byte, so the syndrome of the
// hard decisions of Z^(k-1) is formed there (a share of a three-input XOR of
// the stored bytes per slot pair) instead of in a separate pass over the
// rows.  When it is zero after iteration k, the frame stops with k-1
// iterations and its decisions are read from Z_old, which saturation leaves
// with the sign (and zero) of Z^(k-1).  The exact posteriors of Z^(k-1) are
// gone by then, so a caller asking for them gets the separate check instead.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, gfx9 family
constexpr int kZB = 63;  // bias of the stored Z_old bytes and messages (6-bit)

// Message width b (Sec. V: b = 6..8 bits): extrinsics saturate to Q =
// 2^(b-1) - 1 and the stored Z_old to 2Q (sat_Q(sat_2Q(Z) - L) = sat_Q(Z - L)
// for |L| <= Q).  Z_old and the messages are stored with the same bias ZB, so
// one subtraction of stored values gives Z_old - L.  6 bits: Z_old + 63 in a
// byte (1..125), messages + 63; 7 bits: Z_old + 127 in a byte (1..253),
// messages + 127; 8 bits: Z_old + 127 as int16 (-127..381), messages + 127
// (0..254).  HBIT: the bit of a stored value (plus HADD) that is set exactly
// when Z_old > 0, for the fused hard-decision parity.
template <int QB>
struct Width {
    static constexpr int Q = (1 << (QB - 1)) - 1;
    static constexpr int ZMAX = 2 * Q;
    static constexpr int ZB = QB == 6 ? 63 : 127;
    static constexpr bool Z16 = QB == 8;
    static constexpr uint32_t HADD = QB == 8 ? 0x00800080u : 0u;
    static constexpr uint32_t HMASK = QB == 6 ? 0x00400040u : QB == 7 ? 0x00800080u : 0x01000100u;
    static constexpr uint32_t ZB2 = (uint32_t)ZB * 0x00010001u;
    static constexpr uint32_t ZB4 = (uint32_t)ZB * 0x01010101u;
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// LDS accessed by absolute byte address (the kernel declares only dynamic LDS,
// which starts at address 0): per-edge addresses need no base add.
typedef __attribute__((address_space(3))) uint8_t lds_u8_t;
typedef __attribute__((address_space(3))) uint32_t lds_u32_t;
__device__ __forceinline__ uint32_t lds_byte(uint32_t addr) { return *(lds_u8_t *)(size_t)addr; }
typedef __attribute__((address_space(3))) uint16_t lds_u16_t;
__device__ __forceinline__ uint32_t lds_half(uint32_t addr) { return *(lds_u16_t *)(size_t)addr; }


// The stored Z_old of slot `sl` (Z + ZB) as a signed value, and its store.
template <int QB>
__device__ __forceinline__ int zold_get(const uint8_t *zold, uint32_t sl) {
    if (Width<QB>::Z16) return (int)reinterpret_cast<const int16_t *>(zold)[sl];
    return (int)zold[sl];
}
template <int QB>
__device__ __forceinline__ void zold_put(uint8_t *zold, uint32_t sl, int v) {
    if (Width<QB>::Z16)
        reinterpret_cast<int16_t *>(zold)[sl] = (int16_t)v;
    else
        zold[sl] = (uint8_t)v;
}
// The same read by LDS byte address (the records hold byte addresses).
template <int QB>
__device__ __forceinline__ int zold_at(const uint8_t *lds, uint32_t addr) {
    if (Width<QB>::Z16) return (int)*reinterpret_cast<const int16_t *>(lds + addr);
    return (int)lds[addr];
}
__device__ __forceinline__ void lds_add(uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_add((lds_u32_t *)(size_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ i16x2 as_i(uint32_t v) { return __builtin_bit_cast(i16x2, v); }
__device__ __forceinline__ uint32_t bits(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t bits(i16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// 128 - 256 beta in both 16-bit halves (beta in steps, capped at Q + 1: past
// Q every normalised magnitude is 0 either way; -32640 at Q = 127 still fits)
template <int QB>
__device__ __forceinline__ uint32_t rounding_offset(int b) {
    return (uint32_t)(uint16_t)(int16_t)(128 - 256 * min(b, Width<QB>::Q + 1)) * 0x00010001u;
}

// the same register of the partner lane (lane ^ 1): DPP quad_perm [1,0,3,2]
__device__ __forceinline__ uint32_t partner(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}

// bytes (2s, 2s+1) of w -> the low bytes of the two 16-bit halves
__device__ __forceinline__ uint32_t pair_of(uint32_t w, int s) {
    return __builtin_amdgcn_perm(w, w, s == 0 ? 0x0c010c00u : 0x0c030c02u);
}

// Z_old bytes from the accumulator words, three 10-bit fields per word
// biased by BIAS: four words (twelve slots) per step, one 16-byte LDS read
// and three 4-byte writes.  BIAS is 63 mod 256, so the low byte of a field
// clamped to [BIAS - 62, BIAS + 62] (one v_med3_u32 with constant bounds) is
// the saturated Z_old + 63.  Words past the last one are private padding
// words (read, never used); bytes of slots >= N (unused, the dummy) are left
// untouched.
template <int BIAS, int T>
__device__ __forceinline__ void refresh3(const uint32_t *zacc, uint8_t *zold, int N, int nwords, int tid) {
    constexpr uint32_t lo = BIAS - kZoldMax, hi = BIAS + kZoldMax;
    const int ngroups = (nwords + 3) / 4;
    for (int g = tid; g < ngroups; g += T) {
        const int n0 = g * 12;
        const uint4 v = *reinterpret_cast<const uint4 *>(zacc + 4 * g);
        const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
        uint32_t b[12];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            b[3 * q] = min(max(vw[q] & 1023u, lo), hi);
            b[3 * q + 1] = min(max((vw[q] >> 10) & 1023u, lo), hi);
            b[3 * q + 2] = min(max(vw[q] >> 20, lo), hi);
        }
        if (n0 + 12 <= N) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const uint32_t l = __builtin_amdgcn_perm(b[4 * q + 1], b[4 * q], 0x0c0c0400u);
                const uint32_t h = __builtin_amdgcn_perm(b[4 * q + 3], b[4 * q + 2], 0x04000c0cu);
                *reinterpret_cast<uint32_t *>(zold + n0 + 4 * q) = l | h;
            }
        } else {
            for (int i = 0; i < 12 && n0 + i < N; ++i) zold[n0 + i] = (uint8_t)b[i];
        }
    }
}

// Z_old from the accumulator words with one or two fields per word (PF = 1:
// the word is Z itself; PF = 2: 16-bit fields biased by 32768, i.e. offset
// binary, so flipping each half's top bit gives Z as an int16): four
// variables per step, one 16- or 8-byte LDS read, the clamp to +-ZMAX in
// packed 16-bit halves, and one 4-byte write (8 bytes for the 16-bit Z_old
// of 8-bit messages).  Words past the last one are private padding words
// (read, never used); slots >= N (unused, the dummy) are left untouched.
template <int QB, int PF, int T>
__device__ __forceinline__ void refresh12(const uint32_t *zacc, uint8_t *zold, int N, int nwords, int tid) {
    using Wd = Width<QB>;
    const int ngroups = (nwords * PF + 3) / 4;
    const i16x2 lo = {(short)-Wd::ZMAX, (short)-Wd::ZMAX}, hi = {(short)Wd::ZMAX, (short)Wd::ZMAX};
    const i16x2 zb = {(short)Wd::ZB, (short)Wd::ZB};
    for (int g = tid; g < ngroups; g += T) {
        const int n0 = g * 4;
        uint32_t h[2];  // variables n0, n0+1 and n0+2, n0+3 as Z_old + ZB in 16-bit halves
        if (PF == 1) {
            const uint4 v = *reinterpret_cast<const uint4 *>(zacc + n0);
            // |Z| stays far below 2^15 (the sums are bounded by the field
            // design), so the low halves of the words are Z exactly
            h[0] = __builtin_amdgcn_perm(v.y, v.x, 0x05040100u);
            h[1] = __builtin_amdgcn_perm(v.w, v.z, 0x05040100u);
        } else {
            const uint2 v = *reinterpret_cast<const uint2 *>(zacc + n0 / 2);
            h[0] = v.x ^ 0x80008000u;
            h[1] = v.y ^ 0x80008000u;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
            h[k] = bits(__builtin_elementwise_min(__builtin_elementwise_max(as_i(h[k]), lo), hi) + zb);
        if (n0 + 4 <= N) {
            if (Wd::Z16)
                *reinterpret_cast<uint2 *>(zold + 2 * (size_t)n0) = make_uint2(h[0], h[1]);
            else
                *reinterpret_cast<uint32_t *>(zold + n0) = __builtin_amdgcn_perm(h[1], h[0], 0x06040200u);
        } else {
            for (int k = 0; k < 4 && n0 + k < N; ++k)
                zold_put<QB>(zold, n0 + k, (int)(short)(h[k >> 1] >> (16 * (k & 1))));
        }
    }
}

// Shapes of 1024 threads with at most 8 rows per thread and 7 slots ask for
// 8 waves per SIMD (at most 64 VGPRs): with the small LDS of such codes two
// frames then share a CU, and one frame's barriers hide behind the other's
// work (IRA N=16200, 2048 frames: int8 3.33 -> 2.57 ms, 1-bit 4.04 -> 3.32
// ms; the int8 form spills 16 bytes per thread for it).
template <int D, int R, int T>
constexpr int pk_waves_per_eu() {
    return (T == 1024 && R <= 8 && D <= 7) ? 8 : T == 512 ? 4 : 1;
}

// LANES per row: with 2 the lanes 2u and 2u + 1 hold slots 0..D-1 and
// D..2D-1 of the same two rows, and combine their minima, sign parities and
// syndrome shares with one DPP exchange per row pair.
// One frame decoded by T threads.  LOCK: the workgroup holds several such
// groups that share its barriers (the persistent multi-code kernel), so a
// group whose frame has stopped (or that has no frame: live = false) keeps
// taking part in every barrier until all groups of the workgroup are done.
//  f      frame index in the batch of `a`
//  lds    LDS of the workgroup (address 0: the per-edge records hold absolute
//         LDS addresses, so the kernel declares no LDS but this dynamic
//         array); base: byte offset of this group's region
//  rec_p  the per-edge records of this group's region
//  vote   LOCK: two words of the workgroup's LDS outside every region, and
//         whether this thread is the workgroup's first (it clears them);
//         the workgroup-wide "any group still active" vote goes through them
//         (a library reduction such as __syncthreads_or would add LDS of its
//         own ahead of the dynamic array and move it off address 0)
template <int D, int R, bool ONEBIT, bool FUSED, int T, int LANES, int QB, bool LOCK>
__device__ __forceinline__ void pk_frame(const DecodeArgs &a, int f, bool live, uint8_t *lds, uint32_t base,
                                         const uint32_t *rec_p, int tid, int *vote = nullptr,
                                         bool wg_first = false) {
    static_assert(LANES == 1 || LANES == 2, "one or two lanes per row");
    static_assert(QB == 6 || !ONEBIT, "the 1-bit state holds 6-bit magnitudes");
    using Wd = Width<QB>;
    constexpr int kB = Wd::ZB;  // bias of stored Z_old values and messages
    constexpr int kT = T;  // threads per workgroup (one frame)
    static_assert(R % 2 == 0, "rows are processed in pairs");
    constexpr int RP = R / 2;        // row pairs per thread
    constexpr int W = (D + 1) / 2;   // registers per row pair: two slots (4 bytes) each
    constexpr int NS = (D + 7) / 8;  // 1-bit state registers per row pair: eight slots each
    // B-or-A choice per slot: a mask and a bit-select (the 1-bit state, which
    // keeps the mask as its minimum flag; 8-bit messages, where B can reach
    // 127), else one multiply-add and a max, one instruction fewer per slot
    // pair with the sign (measured 2% faster on the QC code's 11-slot lane
    // pairs as well as on short rows)
    constexpr bool kMaskSelect = ONEBIT || QB == 8;
    const int N = a.c.N;
    const int P = a.zpack;
    const uint32_t dummy = (uint32_t)a.c.dummy;
    uint8_t *zold = lds + base;  // Z_old + 63 at the start of the region (the planner places it there)
    uint32_t *zacc = reinterpret_cast<uint32_t *>(lds + base + a.off_zacc);
    int *flag = reinterpret_cast<int *>(lds + base + a.off_aux);  // [0]: separate check, [1], [2]: fused
    // an idle group (no frame) reads frame 0's input and writes nothing
    const int8_t *__restrict__ z0 = static_cast<const int8_t *>(a.llr_in) + (size_t)(live ? f : 0) * N;
    const __amdgpu_buffer_rsrc_t rec =
        __builtin_amdgcn_make_buffer_rsrc((void *)rec_p, (short)0, RP * D * kT * 16, kRsrcWord3);
    constexpr int NQ = (W + 3) / 4;  // 16-byte shift entries per row pair
    const __amdgpu_buffer_rsrc_t shr =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.c.pk_shift, (short)0, RP * NQ * kT * 16, kRsrcWord3);
    bool done = LOCK && !live;  // LOCK: this group has finished (or never had a frame)
    const int bitsP = (P == 1) ? 32 : (P == 2 ? 16 : 10);
    const int biasP = a.zbias;
    const uint32_t maskP = (P == 1) ? 0xFFFFFFFFu : ((1u << bitsP) - 1u);
    const int nwords = (int)(dummy / (uint32_t)P) + 1;

    const uint32_t *__restrict__ slot_of = a.c.pk_slot;
    // Z_old from the channel LLRs: the loads of kU variables per thread are
    // issued before any of their stores, so the latency of the first touch of
    // z0 (and of the slot table) is paid once per kU variables, not per variable
    constexpr int kU = 8;
    for (int n0 = tid; n0 <= (int)dummy; n0 += kU * kT) {
        int zin[kU];
        uint32_t sl[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {  // unconditional (in-range) loads: no branch between them
            const int nc = min(n0 + u * kT, N - 1);
            zin[u] = (int)z0[nc];
            sl[u] = slot_of[nc];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int n = n0 + u * kT;
            if (n < N)
                zold_put<QB>(zold, sl[u], kB + min(max(zin[u], -Wd::Q), Wd::Q));
            else if (n <= (int)dummy)  // unused slots read as zero; the dummy slot as the largest magnitude
                zold_put<QB>(zold, n, kB + (n == (int)dummy ? Wd::ZMAX : 0));
        }
    }
    __syncthreads();
    for (int w = tid; w < nwords; w += kT) {
        uint32_t v = 0;
        for (int i = 0; i < P; ++i) {
            const int sl = w * P + i;
            const int z = sl < N ? zold_get<QB>(zold, sl) - kB : 0;
            v |= (uint32_t)(z + biasP) << (i * bitsP);
        }
        zacc[w] = v;
    }
    if (tid == 0) {
        flag[0] = 0;
        flag[1] = 0;
        flag[2] = 0;
    }
    if (LOCK && wg_first) {
        vote[0] = 0;
        vote[1] = 0;
    }

    // Message state of each row pair.
    //   int8:  Lw[p][i], bytes 2s / 2s+1: slot 2i+s of rows a / b, as L + 63.
    //   1-bit (Sec. V): St[p][k] for slots j = 8k + i: bit 2i / 16+2i: slot
    //          j held the row minimum in row a / b, so its magnitude is B (A
    //          elsewhere); bit 2i+1 / 17+2i: sign of slot j's own extrinsic t;
    //          Ab[p] bytes: A_a, A_b, B_a, B_b signed by the row's sign
    //          parity, plus 63.  A message is then the stored sign times the
    //          signed A or B, exactly the Sec. V message s_mn f(A, B): the row
    //          parity moves from every per-edge sign bit into the per-row A
    //          and B (s_mn = own sign XOR parity).  The two bits of a slot
    //          index a four-entry byte table per row (+A, +B, -A, -B, plus
    //          63), so one permute rebuilds the old message pair.
    uint32_t Lw[RP][ONEBIT ? 1 : W];
    uint32_t St[RP][NS], Ab[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) {
#pragma unroll
        for (int k = 0; k < NS; ++k) St[p][k] = 0u;
        Ab[p] = 0x3F3F3F3Fu;  // A = B = 0
#pragma unroll
        for (int i = 0; i < (ONEBIT ? 1 : W); ++i) Lw[p][i] = Wd::ZB4;  // L = 0
    }
    __syncthreads();

    const uint32_t tid16 = (uint32_t)tid * 16u;
    uint32_t a8x2 = (uint32_t)a.a8 * 0x00010001u;  // normalisation pair, both 16-bit halves
    uint32_t c8x2 = rounding_offset<QB>(a.b_int);
    // +-64 in both halves, opaque so that the products by it stay multiply-adds
    // (a constant power of two would become a shift and a separate add)
    uint32_t k64 = 0x00400040u, kn64 = 0xFFC0FFC0u;
    asm volatile("" : "+s"(k64), "+s"(kn64));
    // 1-bit table lookup: selector bytes 1 and 3 pick zero, byte 2 the second table
    uint32_t kSelBase = 0x0c040c00u;
    asm volatile("" : "+v"(kSelBase));
    using rec_t = decltype(__builtin_amdgcn_raw_buffer_load_b128(rec, 0u, 0u, 0));
    // one row pair per thread: its records are the same every iteration, so
    // they are loaded once and stay in registers
    constexpr bool KEEP = RP == 1 && !LOCK;
    rec_t rk[KEEP ? D : 1], sk[KEEP ? NQ : 1];
    if constexpr (KEEP) {
#pragma unroll
        for (int j = 0; j < D; ++j) rk[j] = __builtin_amdgcn_raw_buffer_load_b128(rec, tid16, (uint32_t)(j * kT * 16), 0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) sk[q] = __builtin_amdgcn_raw_buffer_load_b128(shr, tid16, (uint32_t)(q * kT * 16), 0);
    }
    // several row pairs per thread: the first pair's records of the next
    // iteration are loaded before the barriers and the refresh, which then
    // hide their latency (not in the 64-register shapes, where the registers
    // would spill)
    constexpr bool PRE = !KEEP && !LOCK && pk_waves_per_eu<D, R, T>() < 8;
    rec_t r0[PRE ? D : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int j = 0; j < D; ++j) r0[j] = __builtin_amdgcn_raw_buffer_load_b128(rec, tid16, (uint32_t)(j * kT * 16), 0);
    }
    int iters = 0;
    bool converged = false;  // the decision of the last completed iteration is a codeword
    bool conv_prev = false;  // FUSED: that of the iteration before the last one is
    for (int it = 1; it <= a.max_iter; ++it) {
        uint32_t it0 = 0;  // opaque zero: keeps the index loads inside the iteration loop
        asm volatile("" : "+s"(it0));
        // FUSED: bits 6 / 22 collect odd hard-decision parities of Z^(it-1)
        // rows; flag[1 + (it & 1)] is set by this iteration and read after its
        // first barrier, the other one (read last iteration) is cleared here
        uint32_t zodd = 0;
        if (FUSED && tid == 0 && !done) flag[1 + ((it + 1) & 1)] = 0;
        if (a.wsched) {  // per-iteration pair (Sec. III's lambda_k, beta_k)
            int a8i, bi;
            sched_pair(a, it, a8i, bi);
            a8x2 = (uint32_t)a8i * 0x00010001u;
            c8x2 = rounding_offset<QB>(bi);
        }
        // (a constant trip count keeps the loop unrolled: the per-row-pair
        // register arrays stay registers)
        if (!(LOCK && done))
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            __builtin_amdgcn_sched_barrier(0);
            // every record of the pair first, in a loop of their own: the slot
            // computations below are then independent of the load order and the
            // scheduler interleaves them, which keeps the dependent packed ops
            // of one slot apart (the 21-slot shape lost most of its hazard
            // wait states this way: int8 12%, 1-bit 21% faster)
            rec_t rc[D], shq[NQ];
#pragma unroll
            for (int j = 0; j < D; ++j)
                rc[j] = KEEP                ? rk[j]
                        : (PRE && p == 0) ? r0[j]
                                          : __builtin_amdgcn_raw_buffer_load_b128(
                                                rec, tid16, it0 + (uint32_t)((p * D + j) * kT * 16), 0);
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                shq[q] = KEEP ? sk[q]
                              : __builtin_amdgcn_raw_buffer_load_b128(shr, tid16,
                                                                      it0 + (uint32_t)((p * NQ + q) * kT * 16), 0);

            uint32_t acc_a[D], acc_b[D], t2[D], lo2[D], mg2[D], h2[D];
            u16x2 min1 = {0xFFFF, 0xFFFF}, min2 = {0xFFFF, 0xFFFF};
            uint32_t Sp[NS], LUTa = 0, LUTb = 0;
#pragma unroll
            for (int k = 0; k < NS; ++k) Sp[k] = ONEBIT ? St[p][k] : 0u;
            if (ONEBIT) {
                // per row, the bytes +A, +B, -A, -B (each plus 63): Ab holds the
                // positive ones; 126 - x negates a biased byte with no borrow
                const uint32_t Nb = 0x7E7E7E7Eu - Ab[p];
                LUTa = __builtin_amdgcn_perm(Nb, Ab[p], 0x06040200u);
                LUTb = __builtin_amdgcn_perm(Nb, Ab[p], 0x07050301u);
            }
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const rec_t r4 = rc[j];
                const uint32_t na = r4[0], nb = r4[1];
                acc_a[j] = r4[2];
                acc_b[j] = r4[3];
                // two loads and one permute: the _d16_hi loads that would fill the
                // high half directly zero the low half on parts with SRAM ECC
                const u16x2 zv = Wd::Z16 ? (u16x2){(unsigned short)lds_half(na), (unsigned short)lds_half(nb)}
                                         : (u16x2){(unsigned short)lds_byte(na), (unsigned short)lds_byte(nb)};
                const uint32_t z2 = bits(zv);
                // FUSED: bit HMASK of the stored value (plus HADD) clear iff
                // Z_old <= 0 (6 bits: Z + 63 <= 63, bit 6)
                if (FUSED) h2[j] = Wd::HADD ? bits(as_u(z2) + as_u(Wd::HADD)) : z2;
                uint32_t l2;
                if (ONEBIT) {
                    // L_old = s * (slot held the minimum ? B : A) + 63 (Eqs. 4-5
                    // inverted): the slot's two bits per row (flag, sign) become
                    // the table index in bytes 0 and 2 of a permute selector
                    // (bytes 1 and 3 select zero), one table per row
                    const unsigned short sh = (unsigned short)(2 * (j & 7));
                    const uint32_t x = bits(as_u(Sp[j >> 3]) >> (u16x2){sh, sh});
                    const uint32_t sel = __builtin_amdgcn_bitop3_b32(x, 0x00030003u, kSelBase, 0xEA);  // (a & b) | c
                    l2 = __builtin_amdgcn_perm(LUTb, LUTa, sel);
                } else {
                    l2 = pair_of(Lw[p][j >> 1], j & 1);
                }
                lo2[j] = l2;
                // Z_old - L_old per row, and its magnitude
                uint32_t tb, mb;
                if constexpr (!Wd::Z16) {
                    // both stored values are non-negative integers below 1024,
                    // which are binary16 subnormals with the same bits: their
                    // binary16 difference is exact and in sign-magnitude form,
                    // so the magnitude is one mask (the sign bits 15 and 31 are
                    // those of the integer difference, +0 for a zero one)
                    tb = __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, z2) - __builtin_bit_cast(f16x2, l2));
                    mb = tb & 0x7FFF7FFFu;
                } else {
                    const i16x2 t = as_i(z2) - as_i(l2);
                    tb = bits(t);
                    mb = bits(__builtin_elementwise_max(t, -t));
                }
                t2[j] = tb;
                const u16x2 mag = as_u(mb);
                mg2[j] = mb;
                min2 = __builtin_elementwise_min(min2, __builtin_elementwise_max(min1, mag));
                min1 = __builtin_elementwise_min(min1, mag);
            }
            // row sign parities (bits 15 and 31), three inputs per XOR
            uint32_t par = t2[0];
#pragma unroll
            for (int j = 1; j + 1 < D; j += 2) par = __builtin_amdgcn_bitop3_b32(par, t2[j], t2[j + 1], 0x96);
            if (D % 2 == 0) par ^= t2[D - 1];
            if (FUSED) {
                uint32_t hp = h2[0];
#pragma unroll
                for (int j = 1; j + 1 < D; j += 2) hp = __builtin_amdgcn_bitop3_b32(hp, h2[j], h2[j + 1], 0x96);
                if (D % 2 == 0) hp ^= h2[D - 1];
                if (LANES == 2) hp ^= partner(hp);
                // bits 6 / 22 of hp: parity of the set bits 6 (Z_old > 0) over
                // the LANES D slots; the hard-decision parity is that plus LANES D
                // (padding slots read the dummy, bit 6 set: they add nothing)
                if ((LANES * D) % 2 == 0)
                    zodd |= hp;
                else
                    zodd = __builtin_amdgcn_bitop3_b32(zodd, hp, 0u, 0xF3);  // a | ~b
            }
            if (LANES == 2) {  // the partner lane holds the other slots of both rows
                const u16x2 o1 = as_u(partner(bits(min1))), o2 = as_u(partner(bits(min2)));
                min2 = __builtin_elementwise_min(__builtin_elementwise_max(min1, o1), __builtin_elementwise_min(min2, o2));
                min1 = __builtin_elementwise_min(min1, o1);
                par ^= partner(par);
            }
            // per row pair: normalised magnitudes of the saturated minima,
            // A, B = max(round(alpha m) - beta, 0) with the offset folded into
            // the rounding constant (128 - 256 beta, beta capped at 32 where A
            // and B are 0 anyway) and an arithmetic shift: the sum stays within
            // +-8064, so the 16-bit halves hold it exactly
            const u16x2 m1 = __builtin_elementwise_min(min1, (u16x2){Wd::Q, Wd::Q});
            const u16x2 m2 = __builtin_elementwise_min(min2, (u16x2){Wd::Q, Wd::Q});
            const i16x2 Am = __builtin_elementwise_max(as_i(bits(m1 * as_u(a8x2) + as_u(c8x2))) >> (i16x2){8, 8},
                                                       (i16x2){0, 0});
            const i16x2 Bm = __builtin_elementwise_max(as_i(bits(m2 * as_u(a8x2) + as_u(c8x2))) >> (i16x2){8, 8},
                                                       (i16x2){0, 0});
            const i16x2 ps = as_i(par) >> (i16x2){15, 15};
            uint32_t B2, A2, mn1, Cs;
            if (kMaskSelect) {  // A and B signed once by the row parity
                B2 = bits((Bm ^ ps) - ps);
                A2 = bits((Am ^ ps) - ps);
                mn1 = bits(min1);
                asm volatile("" : "+v"(B2), "+v"(A2), "+v"(mn1));
            } else {
                // |t_j| equals min1 at the minimum (and at a tie, where A = B)
                // and is at least min1 + 1 elsewhere, where B - 64 (|t_j| - min1)
                // < 0 <= A: so max(A, Cs - 64 |t_j|) with Cs = B + 64 min1 is B
                // at the minimum and A elsewhere (|t_j| <= 93, 189 with 7-bit
                // messages: within 16 bits)
                A2 = bits(Am);
                Cs = bits(min1 * as_u(k64) + as_u(bits(Bm)));
                // +-1.0 in binary16 per half, negative for an odd row parity
                mn1 = (par & 0x80008000u) | 0x3C003C00u;
                asm volatile("" : "+v"(A2), "+v"(Cs), "+v"(mn1));
            }
            uint32_t nl[D];
            uint32_t Sn[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) Sn[k] = 0u;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                i16x2 lb;
                if (kMaskSelect) {
                    // |t_j| >= min1, so (min1 - |t_j|) >> 15 is 0 at the minimum
                    // and -1 elsewhere; one bit-select then picks B or A per row
                    const uint32_t nsel = bits(as_i(bits(as_u(mn1) - as_u(mg2[j]))) >> (i16x2){15, 15});
                    const uint32_t mag = __builtin_amdgcn_bitop3_b32(nsel, A2, B2, 0xCA);  // nsel ? A : B
                    // own sign +-1, then L_new + 63 in one multiply-add
                    const i16x2 sg = (as_i(t2[j]) >> (i16x2){15, 15}) | (i16x2){1, 1};
                    lb = as_i(mag) * sg + (i16x2){kB, kB};
                    // one multiply-add: kept apart from the delta below, which the
                    // compiler would otherwise fold into a multiply and two adds
                    asm volatile("" : "+v"(lb));
                    if (ONEBIT) {  // keep the own-extrinsic sign and the minimum flag
                        const uint32_t sneg = bits(as_i(t2[j]) >> (i16x2){15, 15});
                        uint32_t &S = Sn[j >> 3];
                        S = __builtin_amdgcn_bitop3_b32(sneg, 0x00020002u << (2 * (j & 7)), S, 0xEA);  // (a & b) | c
                        S = __builtin_amdgcn_bitop3_b32(nsel, 0x00010001u << (2 * (j & 7)), S, 0xAE);  // (~a & b) | c
                    }
                } else {
                    const i16x2 mag =
                        __builtin_elementwise_max(as_i(mg2[j]) * as_i(kn64) + as_i(Cs), as_i(A2));
                    // sign +-1.0 per half: own extrinsic's sign (bit 15 of the
                    // sign-magnitude t) XOR the row parity; then L + ZB as one
                    // binary16 multiply-add on subnormals (|L| <= Q < ZB:
                    // exact, and the bits of the result are the integer)
                    const uint32_t sg = (t2[j] & 0x80008000u) ^ mn1;
                    lb = as_i(__builtin_bit_cast(
                        uint32_t, __builtin_elementwise_fma(__builtin_bit_cast(f16x2, bits(mag)),
                                                            __builtin_bit_cast(f16x2, sg),
                                                            __builtin_bit_cast(f16x2, Wd::ZB2))));
                }
                nl[j] = bits(lb);
                const uint32_t d = bits(lb - as_i(lo2[j]));
                const int da = (int)(d << 16) >> 16;
                const int db = (int)d >> 16;
                // word j / 2 holds slots j & ~1 and j | 1, bytes (row a, row b)
                const uint32_t shw = shq[j >> 3][(j >> 1) & 3];
                const uint32_t sha = (shw >> (16 * (j & 1))) & 0xFFu, shb = (shw >> (16 * (j & 1) + 8)) & 0xFFu;
                lds_add(acc_a[j], (uint32_t)da << sha);
                lds_add(acc_b[j], (uint32_t)db << shb);
            }
            if (ONEBIT) {
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    St[p][k] = Sn[k];
                    asm volatile("" : "+v"(St[p][k]));
                }
                // low bytes of the signed halves plus 63: A_a, A_b, B_a, B_b
                Ab[p] = __builtin_amdgcn_perm(bits(as_i(B2) + (i16x2){kZB, kZB}), bits(as_i(A2) + (i16x2){kZB, kZB}),
                                              0x06040200u);
                asm volatile("" : "+v"(Ab[p]));
            } else {
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const uint32_t lo = nl[2 * i];
                    const uint32_t hi = (2 * i + 1 < D) ? nl[2 * i + 1] : Wd::ZB2;
                    Lw[p][i] = __builtin_amdgcn_perm(hi, lo, 0x06040200u);
                    asm volatile("" : "+v"(Lw[p][i]));
                }
            }
        }
        if constexpr (PRE) {
#pragma unroll
            for (int j = 0; j < D; ++j)
                r0[j] = __builtin_amdgcn_raw_buffer_load_b128(rec, tid16, it0 + (uint32_t)(j * kT * 16), 0);
        }
        if (FUSED && it >= 2 && (zodd & Wd::HMASK)) flag[1 + (it & 1)] = 1;
        __syncthreads();
        if (FUSED && it >= 2 && !done && flag[1 + (it & 1)] == 0) {  // Z^(it-1) is a codeword
            conv_prev = true;
            if (!LOCK) break;
            done = true;
        }
        if constexpr (LOCK) {  // every group of the workgroup has finished?
            if (!done && tid == 0) atomicOr(&vote[it & 1], 1);
            __syncthreads();
            const bool any = vote[it & 1] != 0;
            // the other word was last read in the previous iteration, before
            // its second barrier, and is next set after the next first barrier
            if (wg_first) vote[(it + 1) & 1] = 0;
            if (!any) break;
        }
        if (LOCK && done) {
            __syncthreads();
            if (!FUSED && a.early_stop) __syncthreads();
            continue;
        }
        if (tid == 0) *flag = 0;
        if (QB == 6 && P == 3) {
            if (biasP == 319)
                refresh3<319, kT>(zacc, zold, N, nwords, tid);
            else
                refresh3<575, kT>(zacc, zold, N, nwords, tid);
        } else if (P == 1) {
            refresh12<QB, 1, kT>(zacc, zold, N, nwords, tid);
        } else if (P == 2) {
            refresh12<QB, 2, kT>(zacc, zold, N, nwords, tid);
        } else {
            for (int w = tid; w < nwords; w += kT) {
                const uint32_t v = zacc[w];
                for (int i = 0; i < P; ++i) {
                    const int n = w * P + i;
                    if (n < N) {
                        const int z = (P == 1) ? (int)v : (int)((v >> (i * bitsP)) & maskP) - biasP;
                        zold_put<QB>(zold, n, kB + min(max(z, -Wd::ZMAX), Wd::ZMAX));
                    }
                }
            }
        }
        __syncthreads();
        iters = it;
        if (!FUSED && a.early_stop) {
            for (int p = 0; p < RP; ++p) {
                int pa = 0, pb = 0;
                for (int j = 0; j < D; ++j) {
                    const auto r4 = __builtin_amdgcn_raw_buffer_load_b128(
                        rec, tid16, (uint32_t)((p * D + j) * kT * 16), 0);
                    pa ^= zold_at<QB>(lds, r4[0]) <= kB ? 1 : 0;
                    pb ^= zold_at<QB>(lds, r4[1]) <= kB ? 1 : 0;
                }
                if (LANES == 2) {
                    pa ^= (int)partner((uint32_t)pa);
                    pb ^= (int)partner((uint32_t)pb);
                }
                if (pa | pb) atomicOr(flag, 1);
            }
            __syncthreads();
            if (*flag == 0) {
                converged = true;
                if (!LOCK) break;
                done = true;
            }
        }
    }
    int ok = 1;
    // LOCK: every group takes the barriers of the final check; only groups
    // with a frame that has not stopped at a codeword do its work
    const bool check = !converged && !conv_prev && (!LOCK || live);
    if (LOCK || check) {
        __syncthreads();
        if (tid == 0 && check) *flag = 0;
        __syncthreads();
        for (int p = 0; p < RP && check; ++p) {
            int pa = 0, pb = 0;
            for (int j = 0; j < D; ++j) {
                const auto r4 = __builtin_amdgcn_raw_buffer_load_b128(
                    rec, tid16, (uint32_t)((p * D + j) * kT * 16), 0);
                pa ^= zold_at<QB>(lds, r4[0]) <= kB ? 1 : 0;
                pb ^= zold_at<QB>(lds, r4[1]) <= kB ? 1 : 0;
            }
            if (LANES == 2) {
                pa ^= (int)partner((uint32_t)pa);
                pb ^= (int)partner((uint32_t)pb);
            }
            if (pa | pb) atomicOr(flag, 1);
        }
        __syncthreads();
        if (check) ok = (*flag == 0);
    }
    if (LOCK && !live) return;
    // outputs, kU variables per thread and step (slot-table loads first)
    for (int n0 = tid; n0 < N; n0 += kU * kT) {
        uint32_t sl[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) sl[u] = slot_of[min(n0 + u * kT, N - 1)];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int n = n0 + u * kT;
            if (n >= N) continue;
            if (FUSED && conv_prev) {  // decisions of Z^(iters) from its saturated copy
                a.hard_out[(size_t)f * N + n] = zold_get<QB>(zold, sl[u]) <= kB ? 1 : 0;
            } else {
                const uint32_t w = (P == 1) ? sl[u] : (P == 2 ? sl[u] >> 1 : sl[u] / 3u);
                const int i = (int)(sl[u] - w * (uint32_t)P);
                const uint32_t v = zacc[w];
                const int z = (P == 1) ? (int)v : (int)((v >> (i * bitsP)) & maskP) - biasP;
                a.hard_out[(size_t)f * N + n] = z <= 0 ? 1 : 0;
                if (a.llr_out) a.llr_out[(size_t)f * N + n] = (float)((double)z * a.step);
            }
        }
    }
    if (tid == 0) {
        a.iters_out[f] = iters;
        a.ok_out[f] = (uint8_t)ok;
    }
}

// One workgroup per frame.
template <int D, int R, bool ONEBIT, bool FUSED, int T, int LANES, int QB>
__global__ void __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(pk_waves_per_eu<D, R, T>())))
ss_pk_kernel(DecodeArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    pk_frame<D, R, ONEBIT, FUSED, T, LANES, QB, false>(a, blockIdx.x, true, lds, 0u, a.c.pk_idx, threadIdx.x);
}

template <int D, int R, bool ONEBIT, bool FUSED, int T, int S, int QB>
hipError_t launch_one(const DecodeArgs &a, size_t lds, hipStream_t s) {
    auto kern = ss_pk_kernel<D, R, ONEBIT, FUSED, T, S, QB>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_frames), dim3(T), lds, s, a);
    return hipGetLastError();
}

}  // namespace

// Instantiated (slots per lane, rows per thread, threads, lanes per row)
// shapes of the packed kernel (int8 and 1-bit).  Rows of up to 8 slots run
// 1024 threads, or 256 for codes of at most 512 / 1024 checks, so that a CU
// holds several frames; wider rows keep 6 D registers per row pair live, so
// they run 768 threads, whose 3 waves per SIMD leave each wave up to 168
// VGPRs, or split over two lanes (11 slots each) in 512 threads held to 128
// VGPRs, so that two frames share a CU.
#define LDPC_PK_SHAPES(X)   \
    X(6, 2, 256, 1)         \
    X(8, 2, 256, 1)         \
    X(8, 4, 256, 1)         \
    X(6, 2, 1024, 1)        \
    X(6, 4, 1024, 1)        \
    X(7, 8, 1024, 1)        \
    X(7, 16, 1024, 1)       \
    X(7, 32, 1024, 1)       \
    X(8, 8, 1024, 1)        \
    X(8, 16, 1024, 1)       \
    X(8, 32, 1024, 1)       \
    X(21, 4, 768, 1)        \
    X(11, 12, 512, 2)

// Index of a shape in LDPC_PK_SHAPES (compile time).
constexpr int pk_shape_index(int d, int r, int t, int l) {
    int i = 0;
#define X(dd, rr, tt, ll)                             \
    if (d == (dd) && r == (rr) && t == (tt) && l == (ll)) \
        return i;                                     \
    ++i;
    LDPC_PK_SHAPES(X)
#undef X
    return -1;
}
#define PK_SHAPE_ID(d, r, t, l) pk_shape_index(d, r, t, l)

void pk_shapes(int *out, int cap, int *count) {
    int i = 0;
#define X(d, r, t, l)        \
    if (i < cap) {           \
        out[4 * i] = d;      \
        out[4 * i + 1] = r;  \
        out[4 * i + 2] = t;  \
        out[4 * i + 3] = l;  \
    }                        \
    ++i;
    LDPC_PK_SHAPES(X)
#undef X
    *count = i;
}

namespace {
template <int D, int R, int T, int S>
hipError_t launch_shape(const DecodeArgs &a, bool onebit, int qb, size_t lds, hipStream_t s) {
    // the fused check needs at least one iteration and no posterior output
    const bool fused = a.early_stop && a.llr_out == nullptr && a.max_iter >= 1;
    if (onebit) {
        if (qb != 6) return hipErrorInvalidValue;
        return fused ? launch_one<D, R, true, true, T, S, 6>(a, lds, s)
                     : launch_one<D, R, true, false, T, S, 6>(a, lds, s);
    }
    if (qb == 7)
        return fused ? launch_one<D, R, false, true, T, S, 7>(a, lds, s)
                     : launch_one<D, R, false, false, T, S, 7>(a, lds, s);
    if (qb == 8)
        return fused ? launch_one<D, R, false, true, T, S, 8>(a, lds, s)
                     : launch_one<D, R, false, false, T, S, 8>(a, lds, s);
    return fused ? launch_one<D, R, false, true, T, S, 6>(a, lds, s) : launch_one<D, R, false, false, T, S, 6>(a, lds, s);
}
}  // namespace

hipError_t launch_ss_pk(const DecodeArgs &a, int D, int R, int T, int S, bool onebit, int qb, size_t lds,
                        hipStream_t s) {
#define X(d, r, t, l) \
    if (D == d && R == r && T == t && S == l) return launch_shape<d, r, t, l>(a, onebit, qb, lds, s);
    LDPC_PK_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}


// Persistent multi-code decoding: one launch of 1024-thread workgroups, one
// per CU, that take work items from a counter until none is left.  A work
// item is 1024 / T frames of one job (T: the threads of the job's packed
// shape), one frame per group of T threads in its own LDS region, the groups
// sharing the workgroup's barriers (pk_frame with LOCK); items are numbered
// job after job, so the jobs given first (the longest) are taken first.
namespace {

// One work item of shape (D, R, T, LANES): a separate function per shape,
// so that each shape's code keeps its own register allocation (inlined into
// one kernel, the register allocator spilled every shape's code to the
// largest one's budget); the call happens once per work item.
template <int D, int R, bool FUSED, int T, int LANES>
__device__ __noinline__ void pk_item(const PersistJob *J, int item, uint8_t *lds, int *vote, int tid) {
    const int g = tid / T;
    const int f = (item - J->first) * (kPersistThreads / T) + g;
    const DecodeArgs a = J->a;
    pk_frame<D, R, false, FUSED, T, LANES, 6, true>(a, f, f < a.n_frames, lds, (uint32_t)g * J->region,
                                                    J->recs + (size_t)g * J->rec_words, tid % T, vote, tid == 0);
}

template <bool FUSED>
__global__ void __launch_bounds__(kPersistThreads) ss_pk_persist(PersistArgs pa) {
    extern __shared__ __align__(16) uint8_t lds[];
    int *item_sh = reinterpret_cast<int *>(lds + pa.off_item);
    int *vote = item_sh + 1;  // two words after the item word
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) *item_sh = atomicAdd(pa.counter, 1);
        __syncthreads();
        const int item = *item_sh;
        __syncthreads();  // read by every thread before the next item overwrites it
        if (item >= pa.nitems) break;
        int k = 0;
        while (k + 1 < pa.njobs && item >= pa.job[k + 1].first) ++k;
        const PersistJob *J = &pa.job[k];
        switch (J->shape) {
#define X(d, r, t, l)                                                   \
    case PK_SHAPE_ID(d, r, t, l):                                       \
        if constexpr (kPersistThreads % (t) == 0) pk_item<d, r, FUSED, t, l>(J, item, lds, vote, tid); \
        break;
            LDPC_PK_SHAPES(X)
#undef X
        default:
            break;
        }
    }
}

__global__ void zero_counter(int32_t *c) { *c = 0; }

}  // namespace

int pk_shape_id(int D, int R, int T, int S) {
#define X(d, r, t, l) \
    if (D == d && R == r && T == t && S == l) return PK_SHAPE_ID(d, r, t, l);
    LDPC_PK_SHAPES(X)
#undef X
    return -1;
}

hipError_t launch_ss_pk_persist(const PersistArgs &pa, bool fused, size_t lds, int grid, hipStream_t s) {
    auto kern = fused ? ss_pk_persist<true> : ss_pk_persist<false>;
    {  // the records hold absolute LDS addresses: the kernel must have no static LDS
        hipFuncAttributes fa{};
        hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern));
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
    }
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, pa.counter);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPersistThreads), lds, s, pa);
    return hipGetLastError();
}

}  // namespace ldpc
