// Host-side symbolic work for sparse pencils: pattern checks, the union
// pattern of A and B, a reverse Cuthill-McKee ordering and the band widths of
// the reordered pattern.  Values never pass through here: the reordered
// pattern carries, per entry, the index of its value in A's and B's arrays.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace feast_host {

// CSR pattern on the host: row i's column indices are ci[rp[i] .. rp[i+1]).
struct Pattern {
  int64_t n = 0;
  std::vector<int32_t> rp, ci;
};

// Checks rp (n + 1 non-decreasing entries from 0 to nnz) and ci (0 <= col <
// n, no column twice in a row).  Returns an empty string or the first fault.
std::string check_pattern(int64_t n, const int32_t *rp, const int32_t *ci, int64_t nnz);

// Reverse Cuthill-McKee ordering of the symmetrised pattern of P (diagonal
// entries ignored): breadth-first search from a pseudo-peripheral vertex of
// each connected component (lowest degree first, then lowest index), visiting
// neighbours by increasing degree, and the whole order reversed.
// Returns perm with perm[new] = old.
std::vector<int32_t> rcm_order(const Pattern &P);

// The ordering of the sparse path: reverse Cuthill-McKee, or the natural
// order when that is at least as narrow (an already banded pattern can come
// out of reverse Cuthill-McKee wider); kl, ku of the pattern in that order.
std::vector<int32_t> band_order(const Pattern &P, int64_t *kl, int64_t *ku);

// Lower and upper bandwidth of P under the ordering perm (perm[new] = old;
// empty: the identity): the largest new_row - new_col and new_col - new_row.
void band_widths(const Pattern &P, const std::vector<int32_t> &perm, int64_t *kl, int64_t *ku);

// The union pattern of A and B reordered by perm (perm[new] = old), rows in
// new order with columns sorted by their new index; mapA[e] / mapB[e] is the
// index of entry e's value in A's / B's value array, or -1 where that matrix
// has no entry.
struct UnionPattern {
  Pattern P;
  std::vector<int32_t> mapA, mapB;
};
UnionPattern union_reordered(const Pattern &A, const Pattern &B, const std::vector<int32_t> &perm);

}  // namespace feast_host
