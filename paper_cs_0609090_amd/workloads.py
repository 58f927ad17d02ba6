"""Seeded synthetic workloads: parity-check matrices, BPSK/AWGN channel LLRs
and their fixed-point quantisation.

This module only *generates inputs*.  It holds none of the decoder's
arithmetic, so both the CPU oracle (test infrastructure) and the HIP decoder
library can consume what it produces without sharing any method code.

Contents
--------
* ``philox4x32_10`` -- the counter-based generator of Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11), restated from
  its published definition (10 rounds, multipliers 0xD2511F53/0xCD9E8D57,
  Weyl key increments 0x9E3779B9/0xBB67AE85).
* ``awgn_llr`` -- BPSK over AWGN; the channel LLR is 2y/sigma^2 (paper, Sec. II,
  channel model and initial LLR definition).
* ``quantize_llr`` -- 6-bit fixed point held in int8 (step 0.5, clip +-31 steps).
* Code builders with the shapes of the paper's workloads (Sec. I names
  China-HDTV quasi-cyclic irregular codes, DVB-S2 irregular codes and MacKay
  regular codes; none of those tables is reproduced here):
  ``peg_regular`` (progressive edge growth, Hu/Eleftheriou/Arnold 2005),
  ``qc_irregular`` (base matrix of circulant permutations),
  ``ira_code`` (DVB-S2-shaped irregular repeat-accumulate: cyclic column groups
  plus a dual-diagonal parity staircase).
* ``ira_encode`` / ``gf2_nullspace_basis`` -- codewords for tests.

Every builder returns a :class:`ParityCheck` in CSR form (rows are checks,
column indices inside a row in ascending order).
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

__all__ = [
    "ParityCheck", "philox4x32_10", "normals", "awgn_llr", "quantize_llr",
    "ebn0_to_sigma", "peg_regular", "qc_irregular", "ira_code",
    "code_c0_peg1008", "code_c1_qc7493", "code_c2_ira64800", "code_ira16200",
    "ira_encode", "gf2_nullspace_basis", "tree_code", "random_small_code",
    "girth_at_least_6",
]

_MASK32 = np.uint64(0xFFFFFFFF)


# --------------------------------------------------------------------------
# Parity-check container
# --------------------------------------------------------------------------
@dataclasses.dataclass
class ParityCheck:
    """Binary M x N parity-check matrix H in CSR form (paper Sec. II: row m
    lists the variable set N(m))."""

    M: int
    N: int
    row_ptr: np.ndarray  # int32 [M+1]
    col_idx: np.ndarray  # int32 [E]
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def E(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def design_rate(self) -> float:
        return (self.N - self.M) / self.N

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.col_idx, minlength=self.N)

    def dense(self) -> np.ndarray:
        H = np.zeros((self.M, self.N), dtype=np.uint8)
        for m in range(self.M):
            H[m, self.col_idx[self.row_ptr[m]:self.row_ptr[m + 1]]] = 1
        return H

    def syndrome(self, bits: np.ndarray) -> np.ndarray:
        """H x^T mod 2 for x of shape [..., N] (0/1)."""
        b = np.asarray(bits, dtype=np.uint8)
        rows = np.repeat(np.arange(self.M), self.row_degrees())
        out = np.zeros(b.shape[:-1] + (self.M,), dtype=np.uint8)
        np.bitwise_xor.at(out.reshape(-1, self.M).T, rows,
                          b.reshape(-1, self.N)[:, self.col_idx].T)
        return out

    @staticmethod
    def from_rows(M: int, N: int, rows, name: str = "", meta=None) -> "ParityCheck":
        rp = np.zeros(M + 1, dtype=np.int64)
        cols = []
        for m in range(M):
            r = sorted(int(c) for c in rows[m])
            if len(set(r)) != len(r):
                raise ValueError(f"duplicate entry in row {m}")
            cols.extend(r)
            rp[m + 1] = rp[m] + len(r)
        return ParityCheck(M, N, rp.astype(np.int32),
                           np.asarray(cols, dtype=np.int32), name, dict(meta or {}))

    @staticmethod
    def from_dense(H: np.ndarray, name: str = "") -> "ParityCheck":
        H = np.asarray(H) & 1
        return ParityCheck.from_rows(H.shape[0], H.shape[1],
                                     [np.nonzero(H[m])[0] for m in range(H.shape[0])],
                                     name)


# --------------------------------------------------------------------------
# Counter-based RNG and the AWGN channel
# --------------------------------------------------------------------------
def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on arrays of 32-bit counters; returns four
    uint32 arrays.  Restated from Salmon et al. (SC'11)."""
    M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    W0, W1 = 0x9E3779B9, 0xBB67AE85
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in (c0, c1, c2, c3))
    key0, key1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(key0), lo1,
                          hi0 ^ x3 ^ np.uint64(key1), lo0)
        if r != 9:
            key0 = (key0 + W0) & 0xFFFFFFFF
            key1 = (key1 + W1) & 0xFFFFFFFF
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def normals(n_frames: int, n: int, key: tuple[int, int], stream: int = 0,
            frame_offset: int = 0) -> np.ndarray:
    """Standard normals [n_frames, n] in float64.

    Frame f, block i (four values) uses the Philox counter
    (i, frame_offset + f, stream, 0); each pair of 32-bit words gives one
    Box-Muller pair (u = (x + 0.5) / 2^32)."""
    nb = (n + 3) // 4
    i = np.tile(np.arange(nb, dtype=np.uint64), n_frames)
    f = np.repeat(np.arange(n_frames, dtype=np.uint64) + np.uint64(frame_offset), nb)
    w = philox4x32_10(i, f, np.full_like(i, stream), np.zeros_like(i), key[0], key[1])
    u = [(x.astype(np.float64) + 0.5) * (1.0 / 4294967296.0) for x in w]
    r01 = np.sqrt(-2.0 * np.log(u[0]))
    r23 = np.sqrt(-2.0 * np.log(u[2]))
    th01 = 2.0 * math.pi * u[1]
    th23 = 2.0 * math.pi * u[3]
    z = np.stack([r01 * np.cos(th01), r01 * np.sin(th01),
                  r23 * np.cos(th23), r23 * np.sin(th23)], axis=1)
    return z.reshape(n_frames, nb * 4)[:, :n]


def random_bits(n_frames: int, n_bits: int, key: tuple[int, int], stream: int = 0,
                frame_offset: int = 0) -> np.ndarray:
    """Uniform bits [n_frames, n_bits] (uint8): bit b of frame f is bit
    (b mod 32) of word (b mod 128) / 32 of the Philox4x32-10 block for counter
    (b / 128, frame_offset + f, stream, 0)."""
    nb = (n_bits + 127) // 128
    i = np.tile(np.arange(nb, dtype=np.uint64), n_frames)
    f = np.repeat(np.arange(n_frames, dtype=np.uint64) + np.uint64(frame_offset), nb)
    w = philox4x32_10(i, f, np.full_like(i, stream), np.zeros_like(i), key[0], key[1])
    words = np.stack(w, axis=1).reshape(n_frames, nb * 4)          # word order w0..w3 per block
    bits = (words[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1  # bit order 0..31 per word
    return bits.reshape(n_frames, nb * 128)[:, :n_bits].astype(np.uint8)


def ebn0_to_sigma(ebn0_db: float, rate: float) -> float:
    """Noise standard deviation for unit-energy BPSK at code rate R:
    sigma^2 = 1 / (2 R 10^(Eb/N0 / 10))."""
    return math.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0)))


def awgn_llr(N: int, n_frames: int, ebn0_db, rate: float, key=(0x5EED, 0),
             stream: int = 0, codewords: np.ndarray | None = None,
             frame_offset: int = 0) -> np.ndarray:
    """Channel LLRs [n_frames, N] (float32) for BPSK over AWGN.

    Bit 0 maps to +1 (y_n = (-1)^{x_n} + noise) and the LLR is 2y/sigma^2,
    as in Sec. II.  ``ebn0_db`` may be a scalar or one value per frame.
    ``codewords`` defaults to the all-zero word."""
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (n_frames,))
    sigma = np.array([ebn0_to_sigma(float(e), rate) for e in eb])[:, None]
    z = normals(n_frames, N, key, stream, frame_offset)
    if codewords is None:
        x = np.ones((n_frames, N))
    else:
        x = 1.0 - 2.0 * np.asarray(codewords, dtype=np.float64).reshape(n_frames, N)
    y = x + sigma * z
    return (2.0 * y / sigma ** 2).astype(np.float32)


def quantize_llr(llr: np.ndarray, step: float = 0.5, qmax: int = 31) -> np.ndarray:
    """6-bit fixed point in int8: clamp(round_half_away(llr / step), -qmax, qmax)."""
    v = np.asarray(llr, dtype=np.float64) / step
    q = np.sign(v) * np.floor(np.abs(v) + 0.5)
    return np.clip(q, -qmax, qmax).astype(np.int8)


# --------------------------------------------------------------------------
# Code builders
# --------------------------------------------------------------------------
def peg_regular(N: int, M: int, dv: int, dc: int, seed: int, name: str = "") -> ParityCheck:
    """Progressive edge growth (Hu, Eleftheriou, Arnold, IEEE Trans. IT 2005)
    for a (dv, dc)-regular code.

    Variables are processed in order; each new edge of variable v goes to the
    non-full check (degree < dc) farthest from v in the current graph
    (unreached checks count as infinitely far), ties broken by the lowest
    current check degree and then by the seeded generator."""
    if N * dv != M * dc:
        raise ValueError("N*dv must equal M*dc for a regular code")
    rng = np.random.default_rng(seed)
    var_adj: list[list[int]] = [[] for _ in range(N)]
    chk_adj: list[list[int]] = [[] for _ in range(M)]
    cdeg = np.zeros(M, dtype=np.int64)
    INF = 1 << 30
    for v in range(N):
        for k in range(dv):
            dist = np.full(M, INF, dtype=np.int64)
            if var_adj[v]:
                # breadth-first search over the bipartite graph rooted at v
                frontier = list(var_adj[v])
                dist[frontier] = 0
                seen_v = {v}
                depth = 0
                while frontier:
                    depth += 1
                    nxt = []
                    for c in frontier:
                        for u in chk_adj[c]:
                            if u in seen_v:
                                continue
                            seen_v.add(u)
                            for c2 in var_adj[u]:
                                if dist[c2] == INF:
                                    dist[c2] = depth
                                    nxt.append(c2)
                    frontier = nxt
                dist[var_adj[v]] = -1  # never reconnect to an existing neighbour
            open_ = cdeg < dc
            cand = np.nonzero(open_ & (dist >= 0))[0]
            if cand.size == 0:
                raise RuntimeError("PEG ran out of open checks")
            far = dist[cand].max()
            cand = cand[dist[cand] == far]
            low = cdeg[cand].min()
            cand = cand[cdeg[cand] == low]
            c = int(cand[rng.integers(cand.size)]) if cand.size > 1 else int(cand[0])
            var_adj[v].append(c)
            chk_adj[c].append(v)
            cdeg[c] += 1
    return ParityCheck.from_rows(M, N, chk_adj, name or f"peg({N},{M},{dv},{dc})",
                                 {"family": "peg", "seed": seed, "dv": dv, "dc": dc})


def _margin_fill(row_w: np.ndarray, col_w: np.ndarray, rng) -> np.ndarray:
    """0/1 matrix with the given row and column sums (Gale-Ryser greedy):
    columns in random order, each placed on the rows with the largest
    remaining demand (ties broken at random)."""
    R, C = row_w.size, col_w.size
    B = np.zeros((R, C), dtype=np.uint8)
    rem = row_w.astype(np.int64).copy()
    for c in rng.permutation(C):
        w = int(col_w[c])
        key = rem * R * 4 + rng.permutation(R)  # demand first, random tie-break
        rows = np.argsort(-key, kind="stable")[:w]
        if np.any(rem[rows] <= 0):
            raise RuntimeError("margins not realisable")
        B[rows, c] = 1
        rem[rows] -= 1
    if np.any(rem != 0):
        raise RuntimeError("margins not realisable")
    return B


def qc_irregular(mb: int, nb: int, Z: int, row_w_range, col_w_range, seed: int,
                 name: str = "") -> ParityCheck:
    """Quasi-cyclic code from an mb x nb base matrix of Z x Z circulant
    permutations.  Block row weights are drawn in ``row_w_range``, block column
    weights in ``col_w_range`` with the same total; the base pattern is a
    seeded margin-constrained fill; shifts are uniform in [0, Z).

    Entry (b, c) with shift s puts ones at (b*Z + r, c*Z + (r + s) mod Z)."""
    rng = np.random.default_rng(seed)
    rlo, rhi = row_w_range
    clo, chi = col_w_range
    row_w = rng.integers(rlo, rhi + 1, size=mb)
    S = int(row_w.sum())
    col_w = rng.integers(clo, chi + 1, size=nb)
    while col_w.sum() != S:
        c = int(rng.integers(nb))
        if col_w.sum() < S and col_w[c] < min(chi, mb):
            col_w[c] += 1
        elif col_w.sum() > S and col_w[c] > clo:
            col_w[c] -= 1
    base = _margin_fill(row_w, col_w, rng)
    shifts = rng.integers(0, Z, size=(mb, nb))
    M, N = mb * Z, nb * Z
    rows = []
    for b in range(mb):
        cs = np.nonzero(base[b])[0]
        for r in range(Z):
            rows.append(cs * Z + (r + shifts[b, cs]) % Z)
    return ParityCheck.from_rows(M, N, rows, name or f"qc({mb}x{nb},Z={Z})",
                                 {"family": "qc", "seed": seed, "Z": Z,
                                  "base": base, "shifts": np.where(base > 0, shifts, -1)})


def ira_code(N: int, K: int, Q: int, groups: dict[int, int], seed: int,
             name: str = "") -> ParityCheck:
    """DVB-S2-shaped irregular repeat-accumulate code.

    K info columns form K/Q groups of Q columns; ``groups`` maps a column
    degree to the number of groups with that degree.  With q = M/Q, column j
    of a group whose offsets are x_0..x_{d-1} hits rows (x_i + j*q) mod M.
    Offsets are seeded so that every residue class mod q receives the same
    number of entries and no group has two entries in one class; each check
    then carries the same number of info edges.  Parity column K+p hits rows
    p and p+1 (the last one only row M-1): a dual-diagonal staircase."""
    M = N - K
    if K % Q or M % Q:
        raise ValueError("K and M must be multiples of Q")
    q = M // Q
    degs = []
    for d, cnt in sorted(groups.items(), reverse=True):
        degs += [d] * cnt
    if len(degs) * Q != K:
        raise ValueError("group counts do not cover K")
    slots = sum(degs)
    if slots % q:
        raise ValueError("entries do not spread evenly over residue classes")
    per_class = slots // q
    rng = np.random.default_rng(seed)
    # residue-class assignment: each class used per_class times, distinct in a group
    for _attempt in range(1000):
        pool = np.repeat(np.arange(q), per_class)
        rng.shuffle(pool)
        classes, pos, ok = [], 0, True
        for d in degs:
            classes.append(list(pool[pos:pos + d]))
            pos += d
        # repair duplicates inside a group by swapping with other groups
        for g, cl in enumerate(classes):
            for i in range(len(cl)):
                tries = 0
                while cl.count(cl[i]) > 1:
                    tries += 1
                    if tries > 10000:
                        ok = False
                        break
                    h = int(rng.integers(len(classes)))
                    k = int(rng.integers(len(classes[h])))
                    a, b = cl[i], classes[h][k]
                    if h == g or b in cl or a in classes[h]:
                        continue
                    cl[i], classes[h][k] = b, a
                if not ok:
                    break
            if not ok:
                break
        if ok:
            break
    else:
        raise RuntimeError("offset assignment failed")
    offsets = [[int(c) + q * int(rng.integers(Q)) for c in cl] for cl in classes]
    rows: list[list[int]] = [[] for _ in range(M)]
    for g, offs in enumerate(offsets):
        for j in range(Q):
            col = g * Q + j
            for x in offs:
                rows[(x + j * q) % M].append(col)
    for p in range(M):
        rows[p].append(K + p)
        if p + 1 < M:
            rows[p + 1].append(K + p)
    return ParityCheck.from_rows(M, N, rows, name or f"ira({N},{K})",
                                 {"family": "ira", "seed": seed, "Q": Q, "q": q,
                                  "K": K, "offsets": offsets})


def ira_encode(code: ParityCheck, info: np.ndarray) -> np.ndarray:
    """Systematic encoder of an :func:`ira_code` (accumulator over the
    staircase): p_m = p_{m-1} xor (sum of the info bits of row m)."""
    K = code.meta["K"]
    info = np.atleast_2d(np.asarray(info, dtype=np.uint8))
    F = info.shape[0]
    cw = np.zeros((F, code.N), dtype=np.uint8)
    cw[:, :K] = info
    rd = code.row_degrees()
    rows = np.repeat(np.arange(code.M), rd)
    is_info = code.col_idx < K
    acc = np.zeros((F, code.M), dtype=np.uint8)
    np.bitwise_xor.at(acc.T, rows[is_info], info[:, code.col_idx[is_info]].T)
    cw[:, K:] = np.bitwise_xor.accumulate(acc, axis=1)
    return cw


def gf2_nullspace_basis(H: np.ndarray) -> np.ndarray:
    """Basis of {x : H x = 0 mod 2} as rows of a 0/1 matrix (small H only)."""
    A = (np.asarray(H) & 1).astype(np.uint8).copy()
    M, N = A.shape
    pivots = []
    r = 0
    for c in range(N):
        if r >= M:
            break
        nz = np.nonzero(A[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        A[[r, p]] = A[[p, r]]
        others = np.nonzero(A[:, c])[0]
        others = others[others != r]
        A[others] ^= A[r]
        pivots.append(c)
        r += 1
    free = [c for c in range(N) if c not in pivots]
    basis = np.zeros((len(free), N), dtype=np.uint8)
    for i, f in enumerate(free):
        basis[i, f] = 1
        for row, pc in enumerate(pivots):
            basis[i, pc] = A[row, f]
    return basis


def girth_at_least_6(code: ParityCheck) -> bool:
    """True iff no two columns share two rows (no 4-cycles)."""
    seen = set()
    for m in range(code.M):
        cols = code.col_idx[code.row_ptr[m]:code.row_ptr[m + 1]]
        for a in range(len(cols)):
            for b in range(a + 1, len(cols)):
                key = (int(cols[a]), int(cols[b]))
                if key in seen:
                    return False
                seen.add(key)
    return True


def tree_code(n_checks: int, max_dc: int, seed: int) -> ParityCheck:
    """Random code whose Tanner graph is a tree: each new check joins one
    existing variable with 1..max_dc-1 fresh variables."""
    rng = np.random.default_rng(seed)
    rows = []
    N = 0
    for i in range(n_checks):
        fresh = int(rng.integers(1, max_dc))
        if i == 0:
            fresh = max(fresh, 2)
            rows.append(list(range(fresh)))
            N = fresh
        else:
            anchor = int(rng.integers(N))
            rows.append([anchor] + list(range(N, N + fresh)))
            N += fresh
    perm = rng.permutation(N)
    rows = [[int(perm[v]) for v in r] for r in rows]
    order = rng.permutation(n_checks)
    rows = [rows[i] for i in order]
    return ParityCheck.from_rows(n_checks, N, rows, f"tree{seed}")


def random_small_code(M: int, N: int, row_deg_range, seed: int) -> ParityCheck:
    """Random H with row degrees in ``row_deg_range`` (>= 2), cycles allowed."""
    rng = np.random.default_rng(seed)
    lo, hi = row_deg_range
    rows = [rng.choice(N, size=int(rng.integers(lo, hi + 1)), replace=False)
            for _ in range(M)]
    return ParityCheck.from_rows(M, N, rows, f"rand{M}x{N}s{seed}")


# --------------------------------------------------------------------------
# The workload codes (fixed seeds)
# --------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def code_c0_peg1008() -> ParityCheck:
    """Regular (3,6) PEG code, N=1008, M=504, 3024 edges."""
    return peg_regular(1008, 504, 3, 6, seed=0xC0DE0000, name="peg1008")


@functools.lru_cache(maxsize=None)
def code_c1_qc7493() -> ParityCheck:
    """Irregular QC code: 24 x 59 base matrix of 127 x 127 circulants
    (N=7493, M=3048), block column weights 3..11, block row weights 17..21."""
    return qc_irregular(24, 59, 127, (17, 21), (3, 11), seed=0xC0DE0001, name="qc7493")


@functools.lru_cache(maxsize=None)
def code_c2_ira64800() -> ParityCheck:
    """Rate-1/2 IRA code, N=64800, K=32400, 360-column groups (36 of degree 8,
    54 of degree 3), check degree 7 (row 0: 6), E=226799."""
    return ira_code(64800, 32400, 360, {8: 36, 3: 54}, seed=0xC0DE0002, name="ira64800")


@functools.lru_cache(maxsize=None)
def code_ira16200() -> ParityCheck:
    """Rate-1/2 IRA code, N=16200, K=8100, 180-column groups (18 of degree 8,
    27 of degree 3), check degree 7 (row 0: 6), E=56699."""
    return ira_code(16200, 8100, 180, {8: 18, 3: 27}, seed=0xC0DE0003, name="ira16200")
