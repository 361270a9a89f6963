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
    {64, 384, 0, 128, 1},  // ms: nb128_u1 5.79, nb128_u2 5.77, nb128_u3 5.81, nb64_u1 5.96, nb64_u2 5.89, nb64_u3 5.97
    {64, 384, 1, 64, 2},  // ms: nb128_u1 4.35, nb128_u3 4.33, nb64_u1 4.40, nb64_u3 4.25
    {384, 768, 0, 128, 1},  // ms: nb128_u1 18.99, nb128_u2 18.39, nb128_u3 18.95, nb64_u1 19.55, nb64_u2 18.96, nb64_u3 19.66
    {384, 768, 1, 128, 2},  // ms: nb128_u1 12.07, nb128_u3 11.57, nb64_u1 12.95, nb64_u3 11.82
    {768, 1536, 0, 128, 1},  // ms: nb128_u1 62.26, nb128_u2 59.52, nb128_u3 62.77, nb64_u1 66.42, nb64_u2 63.77, nb64_u3 67.07
    {768, 1536, 1, 128, 2},  // ms: nb128_u1 39.15, nb128_u3 36.97, nb64_u1 43.41, nb64_u3 38.45
    {1536, 3072, 0, 128, 1},  // ms: nb128_u1 231.11, nb128_u2 215.22, nb128_u3 231.93, nb64_u1 256.92, nb64_u2 242.31, nb64_u3 259.83
    {1536, 3072, 1, 128, 2},  // ms: nb128_u1 137.39, nb128_u3 124.42, nb64_u1 163.64, nb64_u3 137.70
    {3072, 16385, 0, 128, 1},  // ms: nb128_u1 193.44, nb128_u2 181.09, nb128_u3 194.20, nb64_u1 214.55, nb64_u2 201.97, nb64_u3 215.99
    {3072, 16385, 1, 128, 2},  // ms: nb128_u1 116.02, nb128_u3 106.59, nb64_u1 137.17, nb64_u3 116.56
};

}  // namespace feast_tune
