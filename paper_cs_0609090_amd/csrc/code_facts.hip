// Host-side facts about a parity-check matrix, found once when a handle is
// created and reported by ldpc_code_query (include/ldpc.h): degree
// histograms and the block structure of H, if any.
//
//  - Quasi-cyclic: H is an array of Z x Z blocks, each empty or a circulant
//    permutation (entries (r, (r + s) mod Z) of the block for one shift s).
//  - Repeat-accumulate: the last M columns form a dual-diagonal staircase
//    (column N - M + p hits rows p and p + 1; the last one only row M - 1),
//    and, for the codes of the DVB-S2 tables, the information columns come in
//    cyclic groups of Q columns: column j of a group hits the rows of the
//    group's first column shifted by j * M / Q (mod M).
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "../../include/ldpc.h"
#include "code_facts.h"

namespace ldpc {
namespace {

std::vector<int> divisors_desc(int g) {
    std::vector<int> d;
    for (int k = 1; (int64_t)k * k <= g; ++k)
        if (g % k == 0) {
            d.push_back(k);
            if (k != g / k) d.push_back(g / k);
        }
    std::sort(d.rbegin(), d.rend());
    return d;
}

// H as Z x Z circulant-permutation blocks?
bool is_qc(int M, int N, const int32_t *rp, const int32_t *ci, int Z) {
    const int nbc = N / Z;
    std::vector<int32_t> shift(nbc, -1), count(nbc, 0);
    std::vector<int32_t> touched;
    for (int bi = 0; bi < M / Z; ++bi) {
        touched.clear();
        for (int r = 0; r < Z; ++r) {
            const int m = bi * Z + r;
            for (int e = rp[m]; e < rp[m + 1]; ++e) {
                const int n = ci[e], bj = n / Z, s = ((n % Z) - r + Z) % Z;
                if (count[bj] == 0) {
                    shift[bj] = s;
                    touched.push_back(bj);
                } else if (shift[bj] != s) {
                    return false;
                }
                ++count[bj];
            }
        }
        // a fixed shift and Z entries: every row of the block once (no duplicates in H)
        for (int bj : touched) {
            if (count[bj] != Z) return false;
            count[bj] = 0;
        }
    }
    return true;
}

}  // namespace

void analyse_code(int M, int N, const int32_t *rp, const int32_t *ci, CodeFacts *out) {
    *out = CodeFacts{};
    out->row_hist.assign(65, 0);
    out->col_hist.assign(65, 0);
    std::vector<int32_t> cdeg(N, 0);
    for (int m = 0; m < M; ++m) {
        out->row_hist[std::min(rp[m + 1] - rp[m], 64)]++;
        for (int e = rp[m]; e < rp[m + 1]; ++e) cdeg[ci[e]]++;
    }
    for (int n = 0; n < N; ++n) out->col_hist[std::min(cdeg[n], 64)]++;

    for (int Z : divisors_desc(std::gcd(M, N))) {
        if (Z < 2) break;
        if (is_qc(M, N, rp, ci, Z)) {
            out->structure |= LDPC_STRUCT_QC;
            out->qc_lift = Z;
            break;
        }
    }

    // column lists (rows ascending)
    std::vector<int32_t> cp(N + 1, 0);
    for (int n = 0; n < N; ++n) cp[n + 1] = cp[n] + cdeg[n];
    std::vector<int32_t> crow(rp[M]);
    {
        std::vector<int32_t> fill(cp.begin(), cp.end() - 1);
        for (int m = 0; m < M; ++m)
            for (int e = rp[m]; e < rp[m + 1]; ++e) crow[fill[ci[e]]++] = m;
    }
    const int K = N - M;
    if (K < 0) return;
    bool stair = M >= 1;
    for (int p = 0; p < M && stair; ++p) {
        const int n = K + p;
        if (p + 1 < M)
            stair = cdeg[n] == 2 && crow[cp[n]] == p && crow[cp[n] + 1] == p + 1;
        else
            stair = cdeg[n] == 1 && crow[cp[n]] == p;
    }
    if (!stair) return;
    out->structure |= LDPC_STRUCT_IRA;
    if (K == 0) return;
    std::vector<int32_t> shifted;
    for (int Q : divisors_desc(std::gcd(K, M))) {
        if (Q < 2) break;
        const int q = M / Q;
        bool ok = true;
        for (int n = 0; n < K && ok; ++n) {
            const int first = n - n % Q, j = n % Q;
            if (cdeg[n] != cdeg[first]) {
                ok = false;
                break;
            }
            shifted.assign(crow.begin() + cp[first], crow.begin() + cp[first + 1]);
            for (int32_t &r : shifted) r = (int32_t)(((int64_t)r + (int64_t)j * q) % M);
            std::sort(shifted.begin(), shifted.end());
            ok = std::equal(shifted.begin(), shifted.end(), crow.begin() + cp[n]);
        }
        if (ok) {
            out->structure |= LDPC_STRUCT_IRA_GROUPS;
            out->ira_group = Q;
            break;
        }
    }
}

}  // namespace ldpc
