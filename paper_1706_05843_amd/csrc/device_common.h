// Device-side helpers shared by the hop and network kernels: complex
// arithmetic, precision traits and packed half-field access (layout in
// include/eofa.h: element (rhs, q, s, i) at ((rhs*6 + q)*Vh + i)*Ls + s).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace eofa {

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

template <class T>
struct cx {
  T r, i;
};
template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {  // a*b + c
  return {fma(a.r, b.r, fma(-a.i, b.i, c.r)), fma(a.r, b.i, fma(a.i, b.r, c.i))};
}
template <class T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }  // i a
template <class T>
__device__ __forceinline__ cx<T> cfma_r(T s, cx<T> a, cx<T> c) {  // s*a + c, s real
  return {fma(s, a.r, c.r), fma(s, a.i, c.i)};
}

template <int P>
struct ST;
template <>
struct ST<P64> {
  using R = double;
};
template <>
struct ST<P32> {
  using R = float;
};
template <>
struct ST<P16> {
  using R = float;
};

// ---------------------------------------------------------------------------
// packed field access

struct FD {
  int Ls, Vh, nrhs;
};

// element (r, q, s, i) = r * 6 * Vh * Ls + q * Vh * Ls + (i * Ls + s)
__device__ __forceinline__ size_t qstride(const FD& f) { return (size_t)f.Vh * f.Ls; }
__device__ __forceinline__ size_t eidx(const FD& f, int r, int q, int s, int i) {
  return (size_t)(r * 6 + q) * qstride(f) + (unsigned)(i * f.Ls + s);
}
__device__ __forceinline__ const float* scale_ptr(const void* base, const FD& f) {
  return (const float*)((const char*)base + (size_t)f.nrhs * 6 * qstride(f) * 8);
}
__device__ __forceinline__ size_t sidx(const FD& f, int r, int s, int i) {
  return (size_t)r * qstride(f) + (unsigned)(i * f.Ls + s);
}

template <int P>
__device__ __forceinline__ void ld_pair(const void* base, size_t e, cx<typename ST<P>::R>& a,
                                        cx<typename ST<P>::R>& b) {
  if constexpr (P == P64) {
    const double2* p = (const double2*)base + 2 * e;
    const double2 v0 = p[0], v1 = p[1];
    a = {v0.x, v0.y};
    b = {v1.x, v1.y};
  } else if constexpr (P == P32) {
    const float4 v = ((const float4*)base)[e];
    a = {v.x, v.y};
    b = {v.z, v.w};
  } else {
    const uint2 v = ((const uint2*)base)[e];
    const h2_t h0 = __builtin_bit_cast(h2_t, v.x);
    const h2_t h1 = __builtin_bit_cast(h2_t, v.y);
    a = {(float)h0.x, (float)h0.y};
    b = {(float)h1.x, (float)h1.y};
  }
}

template <int P>
__device__ __forceinline__ void st_pair(void* base, size_t e, cx<typename ST<P>::R> a,
                                        cx<typename ST<P>::R> b) {
  if constexpr (P == P64) {
    double2* p = (double2*)base + 2 * e;
    p[0] = make_double2(a.r, a.i);
    p[1] = make_double2(b.r, b.i);
  } else if constexpr (P == P32) {
    ((float4*)base)[e] = make_float4(a.r, a.i, b.r, b.i);
  } else {
    h2_t h0, h1;
    h0.x = (_Float16)a.r;
    h0.y = (_Float16)a.i;
    h1.x = (_Float16)b.r;
    h1.y = (_Float16)b.i;
    uint2 v;
    v.x = __builtin_bit_cast(unsigned int, h0);
    v.y = __builtin_bit_cast(unsigned int, h1);
    ((uint2*)base)[e] = v;
  }
}

// load pairs [q0, q1) of the spinor at (r, s, i) into v[2*q0 .. 2*q1)
template <int P, class R>
__device__ __forceinline__ void ld_spinor(const void* base, const FD& f, int r, int s, int i, cx<R>* v,
                                          int q0 = 0, int q1 = 6) {
  R sc = R(1);
  if constexpr (P == P16) sc = scale_ptr(base, f)[sidx(f, r, s, i)];
  const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (q < q0 || q >= q1) continue;
    cx<R> a, b;
    ld_pair<P>(base, e0 + q * qs, a, b);
    if constexpr (P == P16) {
      a = sc * a;
      b = sc * b;
    }
    v[2 * q] = a;
    v[2 * q + 1] = b;
  }
}

template <int P, class R>
__device__ __forceinline__ void st_spinor(void* base, const FD& f, int r, int s, int i, const cx<R>* v) {
  if constexpr (P == P16) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].r), fabsf((float)v[c].i)));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cx<float> a = {(float)v[2 * q].r * inv, (float)v[2 * q].i * inv};
      cx<float> b = {(float)v[2 * q + 1].r * inv, (float)v[2 * q + 1].i * inv};
      st_pair<P16>(base, e0 + q * qs, a, b);
    }
    float* sp = (float*)scale_ptr(base, f);
    sp[sidx(f, r, s, i)] = m;
  } else {
    using RS = typename ST<P>::R;
    const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cx<RS> a = {(RS)v[2 * q].r, (RS)v[2 * q].i};
      cx<RS> b = {(RS)v[2 * q + 1].r, (RS)v[2 * q + 1].i};
      st_pair<P>(base, e0 + q * qs, a, b);
    }
  }
}

template <int P>
__device__ __forceinline__ cx<typename ST<P>::R> ld_link(const void* base, size_t j) {
  if constexpr (P == P64) {
    const double2 v = ((const double2*)base)[j];
    return {v.x, v.y};
  } else if constexpr (P == P32) {
    const float2 v = ((const float2*)base)[j];
    return {v.x, v.y};
  } else {
    const h2_t h = __builtin_bit_cast(h2_t, ((const unsigned int*)base)[j]);
    return {(float)h.x, (float)h.y};
  }
}


}  // namespace eofa
