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
    {64, 384, 0, 128, 1},  // ms: nb128_u1 5.72, nb128_u2 5.69, nb128_u3 5.71, nb64_u1 5.87, nb64_u2 5.87, nb64_u3 5.89
    {64, 384, 1, 64, 1},  // ms: nb128_u1 4.47, nb128_u2 4.44, nb128_u3 4.39, nb64_u1 4.38, nb64_u2 4.32, nb64_u3 4.33
    {384, 768, 0, 64, 1},  // ms: nb128_u1 17.95, nb128_u2 17.85, nb128_u3 17.90, nb64_u1 17.95, nb64_u2 17.60, nb64_u3 17.95
    {384, 768, 1, 64, 1},  // ms: nb128_u1 11.72, nb128_u2 11.39, nb128_u3 11.51, nb64_u1 11.86, nb64_u2 10.96, nb64_u3 11.37
    {768, 1536, 0, 64, 1},  // ms: nb128_u1 58.24, nb128_u2 56.98, nb128_u3 58.23, nb64_u1 58.90, nb64_u2 56.61, nb64_u3 59.30
    {768, 1536, 1, 64, 1},  // ms: nb128_u1 37.34, nb128_u2 34.96, nb128_u3 36.11, nb64_u1 38.72, nb64_u2 34.67, nb64_u3 36.35
    {1536, 3072, 0, 128, 1},  // ms: nb128_u1 213.56, nb128_u2 201.03, nb128_u3 212.29, nb64_u1 217.93, nb64_u2 203.08, nb64_u3 218.75
    {1536, 3072, 1, 128, 1},  // ms: nb128_u1 128.49, nb128_u2 112.28, nb128_u3 119.86, nb64_u1 138.14, nb64_u2 116.58, nb64_u3 125.00
    {3072, 16385, 0, 128, 1},  // ms: nb128_u1 177.00, nb128_u2 166.62, nb128_u3 177.14, nb64_u1 180.63, nb64_u2 168.00, nb64_u3 180.79
    {3072, 16385, 1, 128, 1},  // ms: nb128_u1 108.68, nb128_u2 96.90, nb128_u3 102.66, nb64_u1 116.54, nb64_u2 99.41, nb64_u3 106.41
};

}  // namespace feast_tune
