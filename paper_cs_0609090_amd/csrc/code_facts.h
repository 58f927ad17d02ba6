// Host-side facts about a parity-check matrix (degree histograms, block
// structure), found at handle creation for ldpc_code_query.
#pragma once

#include <cstdint>
#include <vector>

namespace ldpc {

struct CodeFacts {
    std::vector<int32_t> row_hist, col_hist;  // 65 bins each (the last: degree >= 64)
    int32_t structure = 0;                    // LDPC_STRUCT_* bits
    int32_t qc_lift = 0;
    int32_t ira_group = 0;
};

// H in CSR form (rows of degree >= 1, no duplicates, indices in range).
void analyse_code(int M, int N, const int32_t *row_ptr, const int32_t *col_idx, CodeFacts *out);

}  // namespace ldpc
