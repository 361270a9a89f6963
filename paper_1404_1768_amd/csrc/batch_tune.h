// Configurations of the batched form's grouped LU, per precision and order
// bucket: the panel width and the loop of the trailing update (feast::GROUP_*).
// Written by `python -m paper_1404_1768_amd.autotune` from factorisation
// timings of every candidate on AMD Radeon Graphics (gfx950:sramecc+:xnack-); entries are looked up with the order
// n* that splits a batch's LU work in half.
#pragma once
#include <cstdint>

namespace feast_tune {

struct Entry {
  int64_t lo, hi;  // bucket: lo <= n* < hi
  int prec;        // FEAST_FP64 or FEAST_MIXED
  int nb;          // panel width, 64 or 128
  int update;      // feast::GROUP_PLAIN, GROUP_UPDATE_M3 or GROUP_UPDATE_PIPE
};

inline constexpr Entry kBatch[] = {
    {64, 384, 0, 128, 0},  // ms: nb128_u1 5.75, nb128_u2 5.75, nb128_u3 5.78, nb64_u1 5.97, nb64_u2 5.91, nb64_u3 6.00
    {64, 384, 1, 64, 2},  // ms: nb128_u1 4.60, nb128_u2 4.31, nb128_u3 4.39, nb64_u1 4.41, nb64_u2 4.27, nb64_u3 4.15
    {384, 768, 0, 128, 1},  // ms: nb128_u1 18.87, nb128_u2 18.13, nb128_u3 18.74, nb64_u1 19.47, nb64_u2 19.00, nb64_u3 19.54
    {384, 768, 1, 128, 1},  // ms: nb128_u1 12.11, nb128_u2 11.35, nb128_u3 11.70, nb64_u1 13.03, nb64_u2 11.46, nb64_u3 11.87
    {768, 1536, 0, 128, 1},  // ms: nb128_u1 62.68, nb128_u2 59.81, nb128_u3 62.68, nb64_u1 66.92, nb64_u2 64.19, nb64_u3 67.45
    {768, 1536, 1, 128, 1},  // ms: nb128_u1 39.24, nb128_u2 35.44, nb128_u3 37.06, nb64_u1 43.73, nb64_u2 36.99, nb64_u3 38.76
    {1536, 3072, 0, 128, 1},  // ms: nb128_u1 232.16, nb128_u2 216.17, nb128_u3 233.19, nb64_u1 262.93, nb64_u2 245.96, nb64_u3 263.01
    {1536, 3072, 1, 128, 1},  // ms: nb128_u1 138.45, nb128_u2 118.66, nb128_u3 126.50, nb64_u1 164.87, nb64_u2 131.86, nb64_u3 139.30
    {3072, 16385, 0, 128, 1},  // ms: nb128_u1 195.93, nb128_u2 182.06, nb128_u3 196.16, nb64_u1 218.06, nb64_u2 203.52, nb64_u3 218.87
    {3072, 16385, 1, 128, 1},  // ms: nb128_u1 117.46, nb128_u2 101.18, nb128_u3 107.90, nb64_u1 138.45, nb64_u2 108.26, nb64_u3 117.97
};

}  // namespace feast_tune
