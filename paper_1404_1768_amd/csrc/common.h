// Shared device-side definitions of the gfx950 FEAST path.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace feast {

// Interleaved complex types: {re, im} as HIP 2-vectors (16 B / 8 B aligned).
using z64 = double2;
using c64 = float2;

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline z64 zmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline z64 zadd(z64 a, z64 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline z64 zsub(z64 a, z64 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline z64 zmul(z64 a, z64 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - b*c
__host__ __device__ inline z64 zfms(z64 a, z64 b, z64 c) {
  return make_double2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
__host__ __device__ inline z64 zconj(z64 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double zabs1(z64 a) { return fabs(a.x) + fabs(a.y); }
// 1 / a by Smith's method (Comm. ACM 5(8), 1962): divide through by the larger
// of |re a|, |im a| first, so no intermediate squares the modulus (|a|^2
// overflows or underflows for |a| beyond about 1e+-154 in FP64 and 1e+-19 in
// FP32, far inside the range of a itself).
__host__ __device__ inline z64 zrecip(z64 a) {
  if (fabs(a.x) >= fabs(a.y)) {
    const double r = a.y / a.x, d = a.x + a.y * r;
    return make_double2(1.0 / d, -r / d);
  }
  const double r = a.x / a.y, d = a.y + a.x * r;
  return make_double2(r / d, -1.0 / d);
}

__host__ __device__ inline c64 cmul(c64 a, c64 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline c64 cfms(c64 a, c64 b, c64 c) {
  return make_float2(a.x - (b.x * c.x - b.y * c.y), a.y - (b.x * c.y + b.y * c.x));
}
__host__ __device__ inline double cabs1(c64 a) { return fabsf(a.x) + fabsf(a.y); }
__host__ __device__ inline c64 crecip(c64 a) {
  if (fabsf(a.x) >= fabsf(a.y)) {
    const float r = a.y / a.x, d = a.x + a.y * r;
    return make_float2(1.0f / d, -r / d);
  }
  const float r = a.x / a.y, d = a.y + a.x * r;
  return make_float2(r / d, -1.0f / d);
}

// Generic complex helpers for templated kernels (T = z64 or c64).
template <typename T> struct cplx_traits;
template <> struct cplx_traits<z64> {
  using real = double;
  __device__ static z64 mul(z64 a, z64 b) { return zmul(a, b); }
  __device__ static z64 fms(z64 a, z64 b, z64 c) { return zfms(a, b, c); }
  __device__ static z64 recip(z64 a) { return zrecip(a); }
  __device__ static double abs1(z64 a) { return zabs1(a); }
  __device__ static z64 make(double r, double i) { return make_double2(r, i); }
};
template <> struct cplx_traits<c64> {
  using real = float;
  __device__ static c64 mul(c64 a, c64 b) { return cmul(a, b); }
  __device__ static c64 fms(c64 a, c64 b, c64 c) { return cfms(a, b, c); }
  __device__ static c64 recip(c64 a) { return crecip(a); }
  __device__ static double abs1(c64 a) { return cabs1(a); }
  __device__ static c64 make(double r, double i) {
    return make_float2(static_cast<float>(r), static_cast<float>(i));
  }
};

// Matrices of a grouped launch.  Matrix b belongs to entry b / nodes (one
// pencil) and is its node b % nodes: order n, leading dimension ld, at
// base + (b % nodes) * stride.  Per-matrix side arrays (pivots, info,
// inverted blocks) stay flat over b with the stride of the largest order.
struct GrpMat {
  void *base;
  int64_t ld, stride, n;
};

template <typename T> struct MatRef {
  T *M;
  int64_t ld, n;
};

// Matrix b of a uniform batch (g == nullptr: base + b * stride, order n) or of
// a grouped one.
template <typename T>
__device__ inline MatRef<T> mat_of(const GrpMat *g, int nodes, T *base, int64_t ld, int64_t stride,
                                   int64_t n, int b) {
  if (g) {
    const GrpMat e = g[b / nodes];
    return {static_cast<T *>(e.base) + (b % nodes) * e.stride, e.ld, e.n};
  }
  return {base + b * stride, ld, n};
}

// Map a linear workgroup id onto a contiguous slice of the work per XCD.
// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs of an
// MI355X; giving each XCD a contiguous range of tiles keeps the tiles that
// share operand panels in the same L2.
__device__ inline int64_t xcd_remap(int64_t id, int64_t total_padded) {
  const int64_t per = total_padded / 8;
  return (id % 8) * per + id / 8;
}

}  // namespace feast
