// Configurations of the batched form's grouped LU, per precision and order
// bucket: the panel width and the loop of the trailing update (feast::GROUP_*).
// Written by `python -m paper_1404_1768_amd.autotune` from factorisation
// timings of every candidate on an MI355X (gfx950); entries are looked up with
// the order n* that splits a batch's LU work in half.
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
    {64, 384, 0, 128, 1},  // ms: nb128_u1 5.89, nb128_u2 5.82, nb128_u3 5.91, nb64_u1 6.01, nb64_u2 6.05, nb64_u3 6.14
    {64, 384, 1, 64, 0},  // ms: nb128_u1 4.05, nb128_u3 4.03, nb64_u1 4.01, nb64_u3 4.11
    {384, 768, 0, 128, 1},  // ms: nb128_u1 19.30, nb128_u2 18.79, nb128_u3 19.52, nb64_u1 20.79, nb64_u2 20.77, nb64_u3 21.20
    {384, 768, 1, 128, 0},  // ms: nb128_u1 11.66, nb128_u3 12.01, nb64_u1 12.23, nb64_u3 12.73
    {768, 1536, 0, 128, 1},  // ms: nb128_u1 64.25, nb128_u2 61.99, nb128_u3 64.49, nb64_u1 74.51, nb64_u2 74.58, nb64_u3 75.77
    {768, 1536, 1, 128, 0},  // ms: nb128_u1 37.14, nb128_u3 37.93, nb64_u1 40.51, nb64_u3 43.36
    {1536, 3072, 0, 128, 1},  // ms: nb128_u1 240.07, nb128_u2 228.32, nb128_u3 242.53, nb64_u1 303.15, nb64_u2 302.24, nb64_u3 308.82
    {1536, 3072, 1, 128, 0},  // ms: nb128_u1 127.60, nb128_u3 133.61, nb64_u1 149.60, nb64_u3 163.80
    {3072, 16385, 0, 128, 1},  // ms: nb128_u1 200.90, nb128_u2 190.11, nb128_u3 201.86, nb64_u1 249.89, nb64_u2 244.82, nb64_u3 253.29
    {3072, 16385, 1, 128, 0},  // ms: nb128_u1 109.58, nb128_u3 113.32, nb64_u1 125.97, nb64_u3 137.54
};

}  // namespace feast_tune
