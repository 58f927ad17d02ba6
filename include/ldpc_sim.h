/*
 * Channel simulation around the decoder: a systematic encoder, random
 * information bits, BPSK over AWGN and per-frame error counts, all on the
 * device, for FER/BER measurement with random codewords.  The decoder does
 * not depend on any of this (Sec. II takes the channel LLRs as its input).
 *
 * Conventions as in ldpc.h: device pointers are HIP device memory on the
 * handle's device (or the current device for the calls without a handle),
 * calls are asynchronous on `stream` (a hipStream_t, NULL = default stream),
 * allocate nothing on the device and never synchronise.  Errors return a
 * status and set ldpc_last_error().
 */
#ifndef LDPC_SIM_H
#define LDPC_SIM_H

#include "ldpc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LDPC_ENC_NONE = 0,
    LDPC_ENC_STAIRCASE = 1, /* the last M columns form the dual-diagonal (accumulator) parity
                               part of an IRA code: column N-M+p has ones in rows p and p+1
                               (the last column: row M-1 only); parities by a running XOR */
    LDPC_ENC_DENSE = 2      /* any other H: Gauss-Jordan elimination over GF(2) on the host,
                               pivot columns taken from the last column down; each parity is
                               the XOR of a fixed set of information bits */
} ldpc_encoder_kind;

/*
 * Describe the systematic encoder of a code, building it on first use (the
 * dense form costs about rank^2 * N / 64 word operations on the host and is
 * refused with LDPC_EUNSUPPORTED above 4e9).  Not for host-only handles'
 * device tables: with device < 0 only the description is built.
 *  kind      out: ldpc_encoder_kind.
 *  k_info    out: K = N - rank(H), the number of information bits.
 *  info_pos  host, N entries, or NULL: the K information columns (ascending)
 *            followed by the N-K parity columns.  A codeword holds bit i of
 *            the information word at column info_pos[i].
 */
ldpc_status ldpc_encoder_info(ldpc_code *code, int32_t *kind, int32_t *k_info, int32_t *info_pos);

/*
 * Encode n_frames information words: codewords[f][info_pos[i]] =
 * info[f][i] and the parity columns chosen so that H c^T = 0 over GF(2).
 *  info       device [F][K] uint8, each 0 or 1 (other values: bit 0 is used).
 *  codewords  device [F][N] uint8 (0/1).
 */
ldpc_status ldpc_encode_batch(ldpc_code *code, int32_t n_frames, const uint8_t *info, uint8_t *codewords,
                              void *stream);

/*
 * Uniform random bits from Philox4x32-10 (Salmon et al., SC'11) with key
 * (key0, key1): bit b of frame f is bit (b mod 32) of word (b mod 128) / 32
 * of the block for counter (b / 128, frame_offset + f, stream_id, 0).
 *  bits  device [F][n_bits] uint8 (0/1).
 */
ldpc_status ldpc_random_bits(int32_t n_frames, int32_t n_bits, uint32_t key0, uint32_t key1,
                             uint32_t stream_id, uint32_t frame_offset, uint8_t *bits, void *stream);

/*
 * BPSK over AWGN (Sec. II): bit c maps to x = 1 - 2c, y = x + sigma_f z and
 * the channel LLR is 2 y / sigma_f^2, all in binary64, rounded once to
 * binary32.  z: values 4i .. 4i+3 of frame f come from the Philox4x32-10
 * block for counter (i, frame_offset + f, stream_id, 0) and key (key0, key1)
 * through Box-Muller on u = (w + 0.5) / 2^32: words (w0, w1) give
 * r cos(2 pi u1), r sin(2 pi u1) with r = sqrt(-2 ln u0), and (w2, w3) the
 * next two.
 *  codewords  device [F][N] uint8 or NULL (the all-zero word).
 *  sigma      device [F] double, > 0 (sigma^2 = 1 / (2 R Eb/N0) for rate R).
 *  llr_f32    device [F][N] float or NULL.
 *  llr_q      device [F][N] int8 or NULL: clamp(round half away from zero of
 *             llr_f32 / step, -qmax, qmax) with step > 0, 1 <= qmax <= 127
 *             (the int8 decoder input: step = llr_step, qmax = 31).
 */
ldpc_status ldpc_channel_awgn(int32_t n_frames, int32_t N, const uint8_t *codewords, const double *sigma,
                              uint32_t key0, uint32_t key1, uint32_t stream_id, uint32_t frame_offset,
                              float *llr_f32, int8_t *llr_q, double step, int32_t qmax, void *stream);

/*
 * bit_errors[f] = number of positions n with (hard[f][n] != 0) !=
 * (codewords[f][n] != 0); NULL codewords stand for the all-zero word.
 *  hard        device [F][N] uint8 (ldpc_decode_batch's hard_out).
 *  bit_errors  device [F] int32.
 */
ldpc_status ldpc_count_errors(int32_t n_frames, int32_t N, const uint8_t *hard, const uint8_t *codewords,
                              int32_t *bit_errors, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_SIM_H */
