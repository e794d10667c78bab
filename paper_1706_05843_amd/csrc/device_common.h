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

// element (r, q, s, i) = r * 6 * Vh * Ls + q * Vh * Ls + (i * Ls + s); FP16S
// groups the components in quads instead (uint4 element (r, j, s, i) at
// r * 3 * Vh * Ls + j * Vh * Ls + (i * Ls + s)): one 16-byte load per lane
// and quad, three per spinor, as many bytes per instruction as FP32 pairs
__device__ __forceinline__ size_t qstride(const FD& f) { return (size_t)f.Vh * f.Ls; }
__device__ __forceinline__ size_t qidx16(const FD& f, int r, int j, int s, int i) {
  return (size_t)(r * 3 + j) * qstride(f) + (unsigned)(i * f.Ls + s);
}
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
  } else {
    static_assert(P == P32, "FP16S fields are read by quads");
    const float4 v = ((const float4*)base)[e];
    a = {v.x, v.y};
    b = {v.z, v.w};
  }
}

template <int P>
__device__ __forceinline__ void st_pair(void* base, size_t e, cx<typename ST<P>::R> a,
                                        cx<typename ST<P>::R> b) {
  if constexpr (P == P64) {
    double2* p = (double2*)base + 2 * e;
    p[0] = make_double2(a.r, a.i);
    p[1] = make_double2(b.r, b.i);
  } else {
    static_assert(P == P32, "FP16S fields are written by quads");
    ((float4*)base)[e] = make_float4(a.r, a.i, b.r, b.i);
  }
}

// the 12 raw half2 words (component c = word c) of an FP16S spinor
__device__ __forceinline__ void ld_words16(const void* base, const FD& f, int r, int s, int i, unsigned* w) {
  const size_t e0 = qidx16(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const uint4 v = ((const uint4*)base)[e0 + j * qs];
    w[4 * j] = v.x;
    w[4 * j + 1] = v.y;
    w[4 * j + 2] = v.z;
    w[4 * j + 3] = v.w;
  }
}

// the spinor at (r, s, i) into v[0..12)
template <int P, class R>
__device__ __forceinline__ void ld_spinor(const void* base, const FD& f, int r, int s, int i, cx<R>* v) {
  if constexpr (P == P16) {
    const R sc = scale_ptr(base, f)[sidx(f, r, s, i)];
    unsigned w[12];
    ld_words16(base, f, r, s, i, w);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const h2_t h = __builtin_bit_cast(h2_t, w[c]);
      v[c] = {sc * (R)(float)h.x, sc * (R)(float)h.y};
    }
  } else {
    const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      cx<R> a, b;
      ld_pair<P>(base, e0 + q * qs, a, b);
      v[2 * q] = a;
      v[2 * q + 1] = b;
    }
  }
}

// Streaming (non-temporal) access for fields touched once per kernel (the
// CG residual and solution): they bypass the cache ways that hold the
// neighbour spinors the hop re-reads.
typedef float f4v_t __attribute__((ext_vector_type(4)));
typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef unsigned u4v_t __attribute__((ext_vector_type(4)));

template <int P, class R>
__device__ __forceinline__ void ld_spinor_nt(const void* base, const FD& f, int r, int s, int i, cx<R>* v) {
  const size_t e0 = P == P16 ? qidx16(f, r, 0, s, i) : eidx(f, r, 0, s, i), qs = qstride(f);
  if constexpr (P == P32) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const f4v_t t = __builtin_nontemporal_load((const f4v_t*)base + e0 + q * qs);
      v[2 * q] = {(R)t.x, (R)t.y};
      v[2 * q + 1] = {(R)t.z, (R)t.w};
    }
  } else if constexpr (P == P64) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const d2v_t* pp = (const d2v_t*)base + 2 * (e0 + q * qs);
      const d2v_t t0 = __builtin_nontemporal_load(pp), t1 = __builtin_nontemporal_load(pp + 1);
      v[2 * q] = {(R)t0.x, (R)t0.y};
      v[2 * q + 1] = {(R)t1.x, (R)t1.y};
    }
  } else {
    const R sc = (R)__builtin_nontemporal_load(scale_ptr(base, f) + sidx(f, r, s, i));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const u4v_t q = __builtin_nontemporal_load((const u4v_t*)base + e0 + j * qs);
      const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const h2_t h = __builtin_bit_cast(h2_t, w[k]);
        v[4 * j + k] = {sc * (R)(float)h.x, sc * (R)(float)h.y};
      }
    }
  }
}

// the raw FP16S words and the site scale of a streamed spinor
__device__ __forceinline__ void ld_raw16_nt(const void* base, const FD& f, int r, int s, int i, float& sc,
                                            unsigned* w) {
  const size_t e0 = qidx16(f, r, 0, s, i), qs = qstride(f);
  sc = __builtin_nontemporal_load(scale_ptr(base, f) + sidx(f, r, s, i));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const u4v_t q = __builtin_nontemporal_load((const u4v_t*)base + e0 + j * qs);
    w[4 * j] = q.x;
    w[4 * j + 1] = q.y;
    w[4 * j + 2] = q.z;
    w[4 * j + 3] = q.w;
  }
}

// FP16S site-spinor: the 12 components as half2 words in units of the
// largest |component|, which is kept as the site's FP32 scale
// Returns the site's |v|^2 as m^2 sum (v/m)^2: the sum over the scaled
// components (each at most 1 + 2^-23) in FP32, the product with m^2 in FP64,
// so no FP32 value overflows (a caller that does not use it pays nothing).
template <bool NT, class R>
__device__ __forceinline__ double st_spinor16(void* base, const FD& f, int r, int s, int i, const cx<R>* v) {
  float m = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf((float)v[c].r), fabsf((float)v[c].i)));
  // hardware reciprocal (1 ulp): the scaled components stay within 1 + 2^-23
  // of the unit, far inside the FP16 range
  const float inv = m > 0.f ? __builtin_amdgcn_rcpf(m) : 0.f;
  unsigned w[12];
  float ns = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const float xr = (float)v[c].r * inv, xi = (float)v[c].i * inv;
    ns = fma(xi, xi, fma(xr, xr, ns));
    h2_t h;
    h.x = (_Float16)xr;
    h.y = (_Float16)xi;
    w[c] = __builtin_bit_cast(unsigned int, h);
  }
  const size_t e0 = qidx16(f, r, 0, s, i), qs = qstride(f);
  float* sp = (float*)scale_ptr(base, f) + sidx(f, r, s, i);
  if constexpr (NT) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const u4v_t q = {w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]};
      __builtin_nontemporal_store(q, (u4v_t*)base + e0 + j * qs);
    }
    __builtin_nontemporal_store(m, sp);
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j)
      ((uint4*)base)[e0 + j * qs] = make_uint4(w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]);
    *sp = m;
  }
  return (double)m * (double)m * (double)ns;
}

template <int P, class R>
__device__ __forceinline__ void st_spinor_nt(void* base, const FD& f, int r, int s, int i, const cx<R>* v) {
  if constexpr (P == P16) {
    st_spinor16<true>(base, f, r, s, i, v);
    return;
  }
  const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
  if constexpr (P == P32) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const f4v_t t = {(float)v[2 * q].r, (float)v[2 * q].i, (float)v[2 * q + 1].r, (float)v[2 * q + 1].i};
      __builtin_nontemporal_store(t, (f4v_t*)base + e0 + q * qs);
    }
  } else if constexpr (P == P64) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      d2v_t* pp = (d2v_t*)base + 2 * (e0 + q * qs);
      const d2v_t t0 = {(double)v[2 * q].r, (double)v[2 * q].i}, t1 = {(double)v[2 * q + 1].r, (double)v[2 * q + 1].i};
      __builtin_nontemporal_store(t0, pp);
      __builtin_nontemporal_store(t1, pp + 1);
    }
  }
}

template <int P, class R>
__device__ __forceinline__ void st_spinor(void* base, const FD& f, int r, int s, int i, const cx<R>* v) {
  if constexpr (P == P16) {
    st_spinor16<false>(base, f, r, s, i, v);
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
