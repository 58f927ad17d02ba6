// Shared pieces of the frames-across-lanes decoders (one frame per lane, 64
// frames per wavefront, frame-minor arrays: element (i, f) at i*Fp + f).
#pragma once

#include "ldpc_internal.h"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace ldpc {
namespace fl {

constexpr int kBlock = kFlThreads;
constexpr int kWaves = kBlock / 64;  // wavefronts per workgroup
constexpr int kNotConverged = INT_MAX;
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, gfx9 family
// Byte offset of the unused slots of a short row or column: every array of a
// chunk is below 2^31 bytes and a lane adds less than that, so the sum stays
// past the end of the buffer without wrapping: loads there return 0 and touch
// no memory, stores are dropped.
constexpr uint32_t kOutOfRange = 0x80000000u;
constexpr int kNonTemporal = 2;  // cache-policy bit of buffer accesses: non-temporal

// The code's index arrays are read-only for the whole call: reading them
// through the constant address space lets wave-uniform loads go to the
// scalar unit (s_load) instead of the vector memory path.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cptr(const T *p) {
    return (const __attribute__((address_space(4))) T *)(p);
}

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWaves + (threadIdx.x >> 6)));
}

// Buffer view of one frame-minor array: every access is a scalar element
// offset (SGPR) plus the lane's frame offset (one VGPR shared by all
// accesses), so no per-access 64-bit address is formed.
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ Buf(const void *p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3)) {}
    __device__ float ldf(uint32_t lane_off, uint32_t elem_off) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, elem_off, 0));
    }
    __device__ void stf(float v, uint32_t lane_off, uint32_t elem_off) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, lane_off, elem_off, 0);
    }
    // non-temporal (streaming) forms: data read or written once per pass, so
    // that it does not push reused data (the posterior gathers) out of the caches
    __device__ float ldf_nt(uint32_t lane_off, uint32_t elem_off) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, elem_off, kNonTemporal));
    }
    __device__ void stf_nt(float v, uint32_t lane_off, uint32_t elem_off) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, lane_off, elem_off, kNonTemporal);
    }
    // V = 1 or 4 consecutive floats per lane (V frames); a 16-byte access
    // moves four times the bytes of a 4-byte one for the same address work.
    // AUX: cache policy (0, or kNonTemporal for streams).
    template <int V, int AUX>
    __device__ void ldv(float (&v)[V], uint32_t lane_off, uint32_t elem_off) const {
        if constexpr (V == 4) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, elem_off, AUX);
            // each component through a scalar: a bit cast of a vector
            // element expression itself reads element 0 with this compiler
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t u = x[c];
                v[c] = __builtin_bit_cast(float, u);
            }
        } else {
            v[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, elem_off, AUX));
        }
    }
    template <int V, int AUX>
    __device__ void stv(const float (&v)[V], uint32_t lane_off, uint32_t elem_off) const {
        if constexpr (V == 4) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 x = {__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1]),
                             __builtin_bit_cast(uint32_t, v[2]), __builtin_bit_cast(uint32_t, v[3])};
            __builtin_amdgcn_raw_buffer_store_b128(x, r, lane_off, elem_off, AUX);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[0]), r, lane_off, elem_off, AUX);
        }
    }
    __device__ int ld8(uint32_t lane_off, uint32_t elem_off) const {  // signed byte
        return (int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(r, lane_off, elem_off, 0);
    }
    __device__ void st8(int v, uint32_t lane_off, uint32_t elem_off) const {
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, lane_off, elem_off, 0);
    }
    __device__ int ld16(uint32_t lane_off, uint32_t elem_off) const {  // signed 16-bit
        return (int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, lane_off, elem_off, 0);
    }
    __device__ void st16(int v, uint32_t lane_off, uint32_t elem_off) const {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, r, lane_off, elem_off, 0);
    }
};

// The kernels below are compiled into every decoder that includes this
// header: internal linkage keeps each copy private to its file.
namespace {

// llr_in [F][N] -> z0 [N][Fp] (frames >= F read as 0), 64x64 tiles via LDS.
template <class T>
__global__ void __launch_bounds__(kBlock) transpose_in(const T *__restrict__ in, T *__restrict__ z0, int N, int F,
                                                       int Fp) {
    __shared__ T tile[64][65];
    const int n0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += kWaves) {
        const int f = f0 + r, n = n0 + tx;
        tile[r][tx] = (f < F && n < N) ? in[(size_t)f * N + n] : (T)0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += kWaves) {
        const int n = n0 + r, f = f0 + tx;
        if (n < N) z0[(size_t)n * Fp + f] = tile[tx][r];
    }
}

// z [N][Fp] -> hard [F][N] (and llr [F][N] = z * step), 64x64 tiles via LDS.
template <class T>
__global__ void __launch_bounds__(kBlock) transpose_out(const T *__restrict__ z, int N, int F, int Fp, double step,
                                                        uint8_t *__restrict__ hard, float *__restrict__ llr) {
    __shared__ T tile[64][65];
    const int n0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += kWaves) {
        const int n = n0 + r;
        tile[r][tx] = n < N ? z[(size_t)n * Fp + f0 + tx] : (T)0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += kWaves) {
        const int f = f0 + r, n = n0 + tx;
        if (f < F && n < N) {
            const T v = tile[tx][r];
            hard[(size_t)f * N + n] = v > (T)0 ? 0 : 1;
            if (llr) llr[(size_t)f * N + n] = std::is_same<T, float>::value ? (float)v : (float)((double)v * step);
        }
    }
}

__global__ void __launch_bounds__(kBlock) init_flags(int32_t *fail, int64_t nfail, int32_t *conv, int Fp) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nfail) fail[i] = 0;
    if (i < Fp) conv[i] = kNotConverged;
}

// Per-frame results from the syndrome flags: iterations (first k >= 1 whose
// syndrome passed when early_stop, else K) and the final syndrome flag.
__global__ void __launch_bounds__(kBlock) frame_out(const int32_t *__restrict__ fail, const int32_t *__restrict__ conv,
                                                    int F, int Fp, int K, int early_stop, int32_t *__restrict__ iters,
                                                    uint8_t *__restrict__ ok) {
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= F) return;
    int it = K;
    if (early_stop) {
        int c = conv[f];
        for (int k = (K >= 2 ? K - 1 : 1); k <= K && c == kNotConverged; ++k)
            if (fail[(size_t)k * Fp + f] == 0) c = k;
        if (c != kNotConverged) it = c;
    }
    iters[f] = it;
    ok[f] = fail[(size_t)K * Fp + f] == 0 ? 1 : 0;
}

// Fold fail[k] into conv (first passing iteration); one wavefront.
__device__ __forceinline__ void fold_conv(int32_t *conv, const int32_t *fail, int k, int Fp, int lane) {
    for (int f = lane; f < Fp; f += 64)
        if (conv[f] == kNotConverged && fail[(size_t)k * Fp + f] == 0) conv[f] = k;
}

}  // namespace

// Chunking: buffer offsets are 32-bit, so every frame-minor array of a chunk
// stays below 2 GiB.  bytes_per_frame_row = the largest array's bytes per
// frame lane (elements x element size).  Returns frames per chunk (a multiple
// of 64), 0 if even one 64-frame group does not fit.
inline int chunk_frames(int64_t bytes_per_frame_row) {
    const int64_t groups = ((int64_t)0x7FFFFF00) / (bytes_per_frame_row * 64);
    return (int)std::min<int64_t>(groups * 64, (int64_t)1 << 30);
}

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Wavefront layout of a strided pass: about 32 wavefronts per CU split over
// the G frame groups; ids past rwaves*G return at once.
inline void wave_layout(int cu_count, int G, int items, int *rwaves, unsigned *grid) {
    const int64_t want = (int64_t)std::max(cu_count, 1) * 32;
    *rwaves = (int)std::max<int64_t>(1, std::min<int64_t>(want / G, std::max(items, 1)));
    *grid = (unsigned)(((int64_t)*rwaves * G + kWaves - 1) / kWaves);
}

}  // namespace fl
}  // namespace ldpc
