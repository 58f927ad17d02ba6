// Channel simulation around the decoder (declared in include/ldpc_sim.h):
// systematic encoder, Philox4x32-10 random bits, BPSK/AWGN channel LLRs and
// per-frame error counts.  Used for FER/BER measurement with random
// codewords; the decoder itself does not depend on it.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ldpc_sim.h"
#include "code_handle.h"
#include "ldpc_internal.h"

namespace {

using ldpc::set_error;

// ---------------------------------------------------------------------------
// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): the round
// multiplies words 0 and 2 by fixed constants and mixes the high halves with
// the other words and the key; the key is bumped by the Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        if (r != 9) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
}

// ---------------------------------------------------------------------------
// Encoder kernels.

// Staircase (IRA accumulator) parity part: s_m = XOR of the information bits
// of row m, parity p_m = s_0 ^ ... ^ s_m (row m: s_m ^ p_{m-1} ^ p_m = 0).
// One workgroup per frame; s in LDS; the prefix XOR is a chunked block scan.
constexpr int kEncThreads = 1024;

__global__ void __launch_bounds__(kEncThreads) enc_staircase(const int32_t *__restrict__ row_ptr,
                                                             const uint32_t *__restrict__ row_ent, int M, int N,
                                                             int K, const uint8_t *__restrict__ info,
                                                             uint8_t *__restrict__ cw) {
    extern __shared__ uint8_t srow[];  // [M]
    __shared__ uint8_t carry[kEncThreads];
    const int tid = threadIdx.x, T = kEncThreads;
    const size_t f = blockIdx.x;
    const uint8_t *u = info + f * (size_t)K;
    uint8_t *c = cw + f * (size_t)N;
    for (int i = tid; i < K; i += T) c[i] = u[i] & 1;
    for (int m = tid; m < M; m += T) {
        uint8_t x = 0;
        for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) {
            const uint32_t col = row_ent[2 * (size_t)e];
            if ((int)col < K) x ^= u[col] & 1;
        }
        srow[m] = x;
    }
    __syncthreads();
    const int chunk = (M + T - 1) / T;
    const int lo = min(M, tid * chunk), hi = min(M, lo + chunk);
    uint8_t x = 0;
    for (int m = lo; m < hi; ++m) x ^= srow[m];
    carry[tid] = x;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {  // inclusive XOR scan of the chunk totals
        const uint8_t v = tid >= d ? carry[tid - d] : 0;
        __syncthreads();
        carry[tid] ^= v;
        __syncthreads();
    }
    x = tid > 0 ? carry[tid - 1] : 0;
    for (int m = lo; m < hi; ++m) {
        x ^= srow[m];
        c[K + m] = x;
    }
}

// Dense parity map: parity r = XOR of the information bits selected by row r
// of the packed map (popcount parity).  One workgroup per frame; the
// information word is packed into LDS first.
constexpr int kDenseThreads = 256;

__global__ void __launch_bounds__(kDenseThreads) enc_dense(const uint32_t *__restrict__ rows, int rank, int words,
                                                           const int32_t *__restrict__ info_pos, int N, int K,
                                                           const uint8_t *__restrict__ info,
                                                           uint8_t *__restrict__ cw) {
    extern __shared__ uint32_t ub[];  // [words]
    const int tid = threadIdx.x, T = kDenseThreads;
    const size_t f = blockIdx.x;
    const uint8_t *u = info + f * (size_t)K;
    uint8_t *c = cw + f * (size_t)N;
    for (int w = tid; w < words; w += T) {
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) {
            const int i = 32 * w + b;
            if (i < K) v |= (uint32_t)(u[i] & 1) << b;
        }
        ub[w] = v;
    }
    __syncthreads();
    for (int i = tid; i < K; i += T) c[info_pos[i]] = u[i] & 1;
    for (int r = tid; r < rank; r += T) {
        const uint32_t *a = rows + (size_t)r * words;
        uint32_t acc = 0;
        for (int w = 0; w < words; ++w) acc ^= (uint32_t)__popc(a[w] & ub[w]);
        c[info_pos[K + r]] = (uint8_t)(acc & 1u);
    }
}

// ---------------------------------------------------------------------------
// Random bits, AWGN channel, error counts.

__global__ void random_bits_kernel(int F, int nbits, uint32_t k0, uint32_t k1, uint32_t sid, uint32_t foff,
                                   uint8_t *__restrict__ bits) {
    const int nb = (nbits + 127) / 128;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)F * nb) return;
    const int f = (int)(t / nb), i = (int)(t % nb);
    uint32_t c[4] = {(uint32_t)i, foff + (uint32_t)f, sid, 0u};
    philox4x32_10(c, k0, k1);
    uint8_t *o = bits + (size_t)f * nbits;
    for (int q = 0; q < 128; ++q) {
        const int b = 128 * i + q;
        if (b < nbits) o[b] = (uint8_t)((c[q >> 5] >> (q & 31)) & 1u);
    }
}

__global__ void awgn_kernel(int F, int N, const uint8_t *__restrict__ cw, const double *__restrict__ sigma,
                            uint32_t k0, uint32_t k1, uint32_t sid, uint32_t foff, float *__restrict__ llr,
                            int8_t *__restrict__ q, double step, int qmax) {
    const int nb = (N + 3) / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)F * nb) return;
    const int f = (int)(t / nb), i = (int)(t % nb);
    uint32_t c[4] = {(uint32_t)i, foff + (uint32_t)f, sid, 0u};
    philox4x32_10(c, k0, k1);
    const double s2p = 1.0 / 4294967296.0;
    const double u0 = ((double)c[0] + 0.5) * s2p, u1 = ((double)c[1] + 0.5) * s2p;
    const double u2 = ((double)c[2] + 0.5) * s2p, u3 = ((double)c[3] + 0.5) * s2p;
    const double twopi = 2.0 * 3.14159265358979323846;
    const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
    const double th01 = twopi * u1, th23 = twopi * u3;
    const double z[4] = {r01 * cos(th01), r01 * sin(th01), r23 * cos(th23), r23 * sin(th23)};
    const double sg = sigma[f];
    const double s2 = sg * sg;
    for (int k = 0; k < 4; ++k) {
        const int n = 4 * i + k;
        if (n >= N) break;
        const size_t o = (size_t)f * N + n;
        const double x = cw ? 1.0 - 2.0 * (double)(cw[o] != 0) : 1.0;
        const double y = x + sg * z[k];
        const float l = (float)((2.0 * y) / s2);
        if (llr) llr[o] = l;
        if (q) {
            const double v = (double)l / step;
            const double a = floor(fabs(v) + 0.5);
            double r = v < 0.0 ? -a : (v > 0.0 ? a : 0.0);
            r = r > (double)qmax ? (double)qmax : (r < -(double)qmax ? -(double)qmax : r);
            q[o] = (int8_t)r;
        }
    }
}

__global__ void __launch_bounds__(256) count_errors_kernel(int N, const uint8_t *__restrict__ hard,
                                                           const uint8_t *__restrict__ cw,
                                                           int32_t *__restrict__ errs) {
    __shared__ int32_t acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    const size_t f = blockIdx.x;
    int n_err = 0;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int h = hard[f * N + n] != 0, b = cw ? cw[f * N + n] != 0 : 0;
        n_err += h != b;
    }
    atomicAdd(&acc, n_err);
    __syncthreads();
    if (threadIdx.x == 0) errs[f] = acc;
}

// ---------------------------------------------------------------------------
// Host: encoder construction.

bool is_staircase(const ldpc_code *c) {
    const int M = c->M, N = c->N, K = N - M;
    if (K < 0) return false;
    std::vector<int32_t> cnt(M, 0);
    std::vector<int32_t> r0(M, -1), r1(M, -1);
    for (int m = 0; m < M; ++m)
        for (int e = c->h_row_ptr[m]; e < c->h_row_ptr[m + 1]; ++e) {
            const int col = c->h_col_idx[e];
            if (col < K) continue;
            const int p = col - K;
            if (cnt[p] == 0) r0[p] = m;
            if (cnt[p] == 1) r1[p] = m;
            ++cnt[p];
        }
    for (int p = 0; p < M; ++p) {
        if (p + 1 < M) {
            if (cnt[p] != 2) return false;
            const int a = std::min(r0[p], r1[p]), b = std::max(r0[p], r1[p]);
            if (a != p || b != p + 1) return false;
        } else if (cnt[p] != 1 || r0[p] != M - 1) {
            return false;
        }
    }
    return true;
}

ldpc_status build_dense(ldpc_code *c, std::vector<uint32_t> &rows_out) {
    const int M = c->M, N = c->N;
    const int W = (N + 63) / 64;
    if ((double)M * M * W > 4e9)
        return set_error(LDPC_EUNSUPPORTED, "dense encoder: elimination too large for this code");
    std::vector<uint64_t> H((size_t)M * W, 0);
    for (int m = 0; m < M; ++m)
        for (int e = c->h_row_ptr[m]; e < c->h_row_ptr[m + 1]; ++e) {
            const int col = c->h_col_idx[e];
            H[(size_t)m * W + col / 64] ^= 1ull << (col % 64);
        }
    // Gauss-Jordan over GF(2), pivot columns from the last one down
    std::vector<int32_t> pivot_col;
    int r = 0;
    for (int col = N - 1; col >= 0 && r < M; --col) {
        const int w = col / 64;
        const uint64_t bit = 1ull << (col % 64);
        int piv = -1;
        for (int i = r; i < M; ++i)
            if (H[(size_t)i * W + w] & bit) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        if (piv != r)
            for (int k = 0; k < W; ++k) std::swap(H[(size_t)piv * W + k], H[(size_t)r * W + k]);
        const uint64_t *pr = &H[(size_t)r * W];
        for (int i = 0; i < M; ++i) {
            if (i == r || !(H[(size_t)i * W + w] & bit)) continue;
            uint64_t *ri = &H[(size_t)i * W];
            for (int k = 0; k < W; ++k) ri[k] ^= pr[k];
        }
        pivot_col.push_back(col);
        ++r;
    }
    const int rank = r, K = N - rank;
    std::vector<char> is_piv(N, 0);
    for (int p : pivot_col) is_piv[p] = 1;
    std::vector<int32_t> info_cols;
    info_cols.reserve(K);
    for (int n = 0; n < N; ++n)
        if (!is_piv[n]) info_cols.push_back(n);
    const int words = std::max(1, (K + 31) / 32);
    rows_out.assign((size_t)rank * words, 0u);
    for (int i = 0; i < rank; ++i)
        for (int t = 0; t < K; ++t) {
            const int col = info_cols[t];
            if (H[(size_t)i * W + col / 64] & (1ull << (col % 64))) rows_out[(size_t)i * words + t / 32] |= 1u << (t % 32);
        }
    c->enc_kind = LDPC_ENC_DENSE;
    c->enc_K = K;
    c->enc_rank = rank;
    c->enc_words = words;
    c->h_info_pos = info_cols;
    c->h_info_pos.insert(c->h_info_pos.end(), pivot_col.begin(), pivot_col.end());
    return LDPC_OK;
}

ldpc_status ensure_encoder(ldpc_code *c) {
    std::lock_guard<std::mutex> lk(c->enc_mu);
    if (c->enc_built) return c->enc_kind == LDPC_ENC_NONE ? set_error(LDPC_EUNSUPPORTED, c->enc_error) : LDPC_OK;
    std::vector<uint32_t> rows;
    if (is_staircase(c)) {
        c->enc_kind = LDPC_ENC_STAIRCASE;
        c->enc_K = c->N - c->M;
        c->enc_rank = c->M;
        c->h_info_pos.resize(c->N);
        for (int n = 0; n < c->N; ++n) c->h_info_pos[n] = n;
    } else {
        const ldpc_status st = build_dense(c, rows);
        if (st != LDPC_OK) {
            c->enc_built = true;
            c->enc_kind = LDPC_ENC_NONE;
            c->enc_error = "dense encoder: elimination too large for this code";
            return st;
        }
    }
    if (c->device >= 0) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(c->device) != hipSuccess) return set_error(LDPC_EDEVICE, "hipSetDevice failed");
        ldpc::reset_alloc_count();
        bool oom = false;
        hipError_t e = ldpc::dev_malloc((void **)&c->d_info_pos, sizeof(int32_t) * c->h_info_pos.size());
        oom = e != hipSuccess;
        if (e == hipSuccess)
            e = hipMemcpy(c->d_info_pos, c->h_info_pos.data(), sizeof(int32_t) * c->h_info_pos.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess && !rows.empty()) {
            e = ldpc::dev_malloc((void **)&c->d_enc_rows, sizeof(uint32_t) * rows.size());
            oom = e != hipSuccess;
            if (e == hipSuccess)
                e = hipMemcpy(c->d_enc_rows, rows.data(), sizeof(uint32_t) * rows.size(), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {  // leave the handle as it was: a later call builds the tables again
            if (c->d_info_pos) (void)hipFree(c->d_info_pos);
            if (c->d_enc_rows) (void)hipFree(c->d_enc_rows);
            c->d_info_pos = nullptr;
            c->d_enc_rows = nullptr;
            (void)hipGetLastError();
        }
        if (prev >= 0) (void)hipSetDevice(prev);
        if (e != hipSuccess)
            return oom ? set_error(LDPC_ENOMEM, "encoder tables: device allocation failed")
                       : set_error(LDPC_EDEVICE, "encoder tables: copy to the device failed");
    }
    c->enc_built = true;
    return LDPC_OK;
}

struct DeviceScope {
    int prev = -1;
    bool ok = true;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

ldpc_status ldpc_encoder_info(ldpc_code *code, int32_t *kind, int32_t *k_info, int32_t *info_pos) {
    if (!code) return set_error(LDPC_EINVAL, "code is NULL");
    const ldpc_status st = ensure_encoder(code);
    if (st != LDPC_OK) return st;
    if (kind) *kind = code->enc_kind;
    if (k_info) *k_info = code->enc_K;
    if (info_pos) std::copy(code->h_info_pos.begin(), code->h_info_pos.end(), info_pos);
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_encode_batch(ldpc_code *code, int32_t n_frames, const uint8_t *info, uint8_t *codewords,
                              void *stream) {
    if (!code) return set_error(LDPC_EINVAL, "code is NULL");
    if (n_frames < 0) return set_error(LDPC_EINVAL, "n_frames < 0");
    if (code->device < 0) return set_error(LDPC_EINVAL, "host-only handle (device < 0) cannot encode");
    const ldpc_status st = ensure_encoder(code);
    if (st != LDPC_OK) return st;
    if (n_frames == 0) return LDPC_OK;
    if (!codewords || (!info && code->enc_K > 0)) return set_error(LDPC_EINVAL, "info and codewords are required");
    DeviceScope g(code->device);
    if (!g.ok) return set_error(LDPC_EDEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (code->enc_kind == LDPC_ENC_STAIRCASE) {
        const size_t lds = (size_t)code->M;
        if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void *>(enc_staircase),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return set_error(LDPC_EUNSUPPORTED, "staircase encoder: M exceeds the LDS of one workgroup");
        hipLaunchKernelGGL(enc_staircase, dim3((unsigned)n_frames), dim3(kEncThreads), lds, s, code->d_row_ptr,
                           code->d_row_ent, code->M, code->N, code->enc_K, info, codewords);
    } else {
        const size_t lds = sizeof(uint32_t) * (size_t)code->enc_words;
        if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void *>(enc_dense),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return set_error(LDPC_EUNSUPPORTED, "dense encoder: information word exceeds the LDS of one workgroup");
        hipLaunchKernelGGL(enc_dense, dim3((unsigned)n_frames), dim3(kDenseThreads), lds, s, code->d_enc_rows,
                           code->enc_rank, code->enc_words, code->d_info_pos, code->N, code->enc_K, info,
                           codewords);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("encoder launch failed: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_random_bits(int32_t n_frames, int32_t n_bits, uint32_t key0, uint32_t key1, uint32_t stream_id,
                             uint32_t frame_offset, uint8_t *bits, void *stream) {
    if (n_frames < 0 || n_bits < 0) return set_error(LDPC_EINVAL, "n_frames or n_bits < 0");
    if ((int64_t)n_frames * n_bits == 0) return LDPC_OK;
    if (!bits) return set_error(LDPC_EINVAL, "bits is NULL");
    const int64_t threads = (int64_t)n_frames * ((n_bits + 127) / 128);
    hipLaunchKernelGGL(random_bits_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n_frames, n_bits, key0, key1, stream_id, frame_offset, bits);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_channel_awgn(int32_t n_frames, int32_t N, const uint8_t *codewords, const double *sigma,
                              uint32_t key0, uint32_t key1, uint32_t stream_id, uint32_t frame_offset,
                              float *llr_f32, int8_t *llr_q, double step, int32_t qmax, void *stream) {
    if (n_frames < 0 || N < 0) return set_error(LDPC_EINVAL, "n_frames or N < 0");
    if (llr_q && !(step > 0.0 && std::isfinite(step))) return set_error(LDPC_EINVAL, "step must be > 0");
    if (llr_q && (qmax < 1 || qmax > 127)) return set_error(LDPC_EINVAL, "qmax outside [1, 127]");
    if ((int64_t)n_frames * N == 0) return LDPC_OK;
    if (!sigma || (!llr_f32 && !llr_q)) return set_error(LDPC_EINVAL, "sigma and an output are required");
    const int64_t threads = (int64_t)n_frames * ((N + 3) / 4);
    hipLaunchKernelGGL(awgn_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n_frames, N, codewords, sigma, key0, key1, stream_id,
                       frame_offset, llr_f32, llr_q, step, qmax);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

ldpc_status ldpc_count_errors(int32_t n_frames, int32_t N, const uint8_t *hard, const uint8_t *codewords,
                              int32_t *bit_errors, void *stream) {
    if (n_frames < 0 || N < 0) return set_error(LDPC_EINVAL, "n_frames or N < 0");
    if (n_frames == 0) return LDPC_OK;
    if (!hard || !bit_errors) return set_error(LDPC_EINVAL, "hard and bit_errors are required");
    hipLaunchKernelGGL(count_errors_kernel, dim3((unsigned)n_frames), dim3(256), 0, static_cast<hipStream_t>(stream),
                       N, hard, codewords, bit_errors);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LDPC_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
    ldpc::clear_error();
    return LDPC_OK;
}

}  // extern "C"
