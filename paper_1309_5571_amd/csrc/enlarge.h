// The enlarged-block basis shared by dmrg_enlarge and the l-1-1-r plans.
//
// An enlarged block slow (x) fast (Alg. 1, steps 1-2: a block and its
// neighbouring site, L = l (x) s1 or R = s2 (x) r) has one sector per label
// sum q = q_slow + q_fast that holds states, in ascending lexicographic order.
// Inside sector q the combinations (s_slow, s_fast) follow in ascending order
// of s_slow, each a row-major [d(s_slow)][d(s_fast)] sub-block (slow index
// first, the order of the Kronecker product slow (x) fast).
#pragma once

#include <cstdint>
#include <vector>

#include "dmrg.h"

namespace dmrg {

struct Combo {
    int32_t s, f;  // slow sector, fast sector
    int64_t off;   // first state of the sub-block inside the enlarged sector
};

struct Enlarged {
    int rank = 1;
    std::vector<int32_t> label;                // [nsec * rank], ascending
    std::vector<int64_t> dim;                  // [nsec], > 0
    std::vector<std::vector<Combo>> combos;    // per sector, ascending s
    std::vector<std::vector<int32_t>> where;   // [nslow][nfast] -> sector, -1 if the product is empty
    std::vector<std::vector<int64_t>> at;      // [nslow][nfast] -> offset inside that sector
    int nsec() const { return (int)dim.size(); }
    int find(const int32_t *lab) const;        // sector with this label, -1 if none
    dmrg_space space() const { return dmrg_space{nsec(), rank, label.data(), dim.data()}; }
};

// Requires valid spaces of the same rank (labels ascending).
Enlarged enlarged_space(const dmrg_space &slow, const dmrg_space &fast);

// One block of an operator whose data are in host memory, as a dense
// row-major [rows = dim(dst)][cols = dim(src)] matrix (identity and diagonal
// operators give one square block per sector).
struct HostBlock {
    int32_t src, dst;
    int64_t rows, cols;
    std::vector<double> m;
};
std::vector<HostBlock> host_blocks(const dmrg_space &sp, const dmrg_op &op);

}  // namespace dmrg
