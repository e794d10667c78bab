// Kernels of the gauge-covariant parallel-transport network (flexible
// preconditioner) and of flexible CG. Not part of the paper's method: the
// layer form, loss and optimiser are this library's choices.
//
// Layer C_in -> C_out on every s-slice, output parity p:
//   y_c(x) = sum_t sum_c' W[t][c][c'] (T_t X_c')(x),
//   T_0 = 1, T_{1+mu} psi(x) = U_mu(x) psi(x+mu), T_{5+mu} psi(x) = U_mu(x-mu)^dag psi(x-mu)
// (boundary phases included: the per-parity links of the hop kernels are
// exactly these transports). Activations are packed FP32 half-fields with
// the channel as the right-hand-side index. Weights: bfloat16 pairs
// (re, im) [9][C_out][C_in], FP32 arithmetic.
// Adjoint in X: conj(W[swap t][c][c']) with T_{+mu}^dag = T_{-mu} (swap t).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "internal.h"
#include "nn_internal.h"

namespace eofa {

__device__ __forceinline__ float bf16_to_f32(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ unsigned short f32_to_bf16(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ int swap_term(int t) { return t == 0 ? 0 : (t <= 4 ? t + 4 : t - 4); }

// z <- L z for a 12-component spinor (colour matvec per spin), L = 9 complex
__device__ __forceinline__ void link_mul(const float2* L, cx<float>* z) {
  cx<float> U[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) U[k] = {L[k].x, L[k].y};
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    const cx<float> a = z[sp * 3], b = z[sp * 3 + 1], c = z[sp * 3 + 2];
#pragma unroll
    for (int r = 0; r < 3; ++r) z[sp * 3 + r] = cfma(U[r * 3 + 2], c, cfma(U[r * 3 + 1], b, cmul(U[r * 3], a)));
  }
}

// One thread: one 5D site (i, s) of the output parity and a block of CB
// output channels c0 .. c0+CB-1. For each stencil term t the input channels
// are mixed first (z_c = sum_c' W[t][c][c'] X_c'(neighbour)) and the CB mixed
// spinors are then transported (one link product per term and channel), so
// every input spinor is loaded once per channel block.
constexpr int NET_CB = 4;

template <bool ADJ>
__global__ void __launch_bounds__(256) pt_layer_kernel(NetLayerArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int c0 = blockIdx.y * NET_CB;
  if (idx >= a.Vh * a.Ls) return;
  const int i = idx / a.Ls, s = idx - i * a.Ls;
  const int p = a.parity;
  const int nco = min(NET_CB, a.Cout - c0);
  const FD fin = {a.Ls, a.Vh, a.Cin};
  cx<float> acc[NET_CB][12];
#pragma unroll
  for (int cc = 0; cc < NET_CB; ++cc)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[cc][k] = {0.f, 0.f};
  for (int t = 0; t < 9; ++t) {
    const int j = t == 0 ? i : a.nbr[(size_t)i * 8 + t - 1];
    const float* src = a.xin[t == 0 ? p : 1 - p];
    cx<float> z[NET_CB][12];
#pragma unroll
    for (int cc = 0; cc < NET_CB; ++cc)
#pragma unroll
      for (int k = 0; k < 12; ++k) z[cc][k] = {0.f, 0.f};
    for (int ci = 0; ci < a.Cin; ++ci) {
      cx<float> v[12];
      ld_spinor<P32>(src, fin, ci, s, j, v);
#pragma unroll
      for (int cc = 0; cc < NET_CB; ++cc) {
        if (cc >= nco) break;
        const int c = c0 + cc;
        size_t k;
        float wr, wi;
        if (!ADJ) {
          k = (((size_t)t * a.Cout + c) * a.Cin + ci) * 2;
          wr = bf16_to_f32(a.w[k]);
          wi = bf16_to_f32(a.w[k + 1]);
        } else {  // forward layer had C_out = a.Cin, C_in = a.Cout
          k = (((size_t)swap_term(t) * a.Cin + ci) * a.Cout + c) * 2;
          wr = bf16_to_f32(a.w[k]);
          wi = -bf16_to_f32(a.w[k + 1]);
        }
        const cx<float> w = {wr, wi};
#pragma unroll
        for (int q = 0; q < 12; ++q) z[cc][q] = cfma(w, v[q], z[cc][q]);
      }
    }
#pragma unroll
    for (int cc = 0; cc < NET_CB; ++cc) {
      if (cc >= nco) break;
      if (t > 0) link_mul((const float2*)a.links + ((size_t)i * 8 + t - 1) * 9, z[cc]);
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[cc][q] = acc[cc][q] + z[cc][q];
    }
  }
  const FD fo = {a.Ls, a.Vh, a.Cout};
#pragma unroll
  for (int cc = 0; cc < NET_CB; ++cc) {
    if (cc >= nco) break;
    st_spinor<P32>(a.yout, fo, c0 + cc, s, i, acc[cc]);
  }
}

// dL/dW*[t][c][ci] partial sums: sum over sites of G_c(x) . conj((T_t X_ci)(x)).
// Work-group (blk, t*ncb + cb, parity): term t, output channels
// cb*NET_CB .. +NET_CB-1, all input channels; each thread loads its site's
// G_c once and each transported input once per channel block.
__global__ void __launch_bounds__(256) pt_wgrad_kernel(NetGradArgs a) {
  const int ncb = (a.Cout + NET_CB - 1) / NET_CB;
  const int t = blockIdx.y / ncb, cb = blockIdx.y - t * ncb;
  const int c0 = cb * NET_CB;
  const int nco = min(NET_CB, a.Cout - c0);
  const int p = blockIdx.z;
  const FD fx = {a.Ls, a.Vh, a.Cin}, fg = {a.Ls, a.Vh, a.Cout};
  float ar[NET_CB][NET_MAXC], ai[NET_CB][NET_MAXC];
#pragma unroll
  for (int cc = 0; cc < NET_CB; ++cc)
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci) ar[cc][ci] = ai[cc][ci] = 0.f;
  const int n = a.Vh * a.Ls;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    const int i = idx / a.Ls, s = idx - i * a.Ls;
    const int j = t == 0 ? i : a.nbr[p][(size_t)i * 8 + t - 1];
    cx<float> g[NET_CB][12];
#pragma unroll
    for (int cc = 0; cc < NET_CB; ++cc) {
      if (cc >= nco) break;
      ld_spinor<P32>(a.g[p], fg, c0 + cc, s, i, g[cc]);
    }
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci) {
      if (ci >= a.Cin) break;
      cx<float> v[12];
      ld_spinor<P32>(a.x[t == 0 ? p : 1 - p], fx, ci, s, j, v);
      if (t > 0) link_mul((const float2*)a.links[p] + ((size_t)i * 8 + t - 1) * 9, v);
#pragma unroll
      for (int cc = 0; cc < NET_CB; ++cc) {
        if (cc >= nco) break;
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int q = 0; q < 12; ++q) {  // g * conj(v)
          sr = fmaf(g[cc][q].r, v[q].r, fmaf(g[cc][q].i, v[q].i, sr));
          si = fmaf(g[cc][q].i, v[q].r, fmaf(-g[cc][q].r, v[q].i, si));
        }
        ar[cc][ci] += sr;
        ai[cc][ci] += si;
      }
    }
  }
  // reduce the NET_CB x C_in complex sums over the work-group
  __shared__ double red[4][2 * NET_CB * NET_MAXC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cc = 0; cc < NET_CB; ++cc)
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci) {
      if (cc >= nco || ci >= a.Cin) continue;
      double vr = ar[cc][ci], vi = ai[cc][ci];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        vr += __shfl_xor(vr, off, 64);
        vi += __shfl_xor(vi, off, 64);
      }
      if (lane == 0) {
        red[wv][2 * (cc * NET_MAXC + ci)] = vr;
        red[wv][2 * (cc * NET_MAXC + ci) + 1] = vi;
      }
    }
  __syncthreads();
  const int k = threadIdx.x;  // (cc, ci, comp)
  if (k < 2 * NET_CB * NET_MAXC) {
    const int comp = k & 1, cc = (k >> 1) / NET_MAXC, ci = (k >> 1) % NET_MAXC;
    if (cc < nco && ci < a.Cin) {
      double tsum = 0.0;
      for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w][k];
      const int y = t * a.Cin + ci, c = c0 + cc;
      a.partial[((((size_t)y * 2 + p) * a.Cout + c) * gridDim.x + blockIdx.x) * 2 + comp] = tsum;
    }
  }
}

// gW[t][c][ci] (+)= sum over parity and blocks (fixed order), as (re, im) doubles
__global__ void pt_wgrad_final(const double* partial, int Cin, int Cout, int nblk, int accumulate, double* gw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // over 9*Cout*Cin*2
  if (k >= 9 * Cout * Cin * 2) return;
  const int comp = k & 1, rest = k >> 1;
  const int ci = rest % Cin, c = (rest / Cin) % Cout, t = rest / (Cin * Cout);
  const int y = t * Cin + ci;
  double s = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < nblk; ++b) s += partial[((((size_t)y * 2 + p) * Cout + c) * nblk + b) * 2 + comp];
  gw[k] = accumulate ? gw[k] + s : s;
}

// loss seed: G = (y - e)/|e|^2 on the odd sites; partial |y - e|^2
__global__ void __launch_bounds__(256) net_loss_kernel(int Vh, int Ls, const float* y, const float* e, float* g,
                                                       const double* enorm, double* partial) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  double d2 = 0.0;
  if (idx < Vh * Ls) {
    const int i = idx / Ls, s = idx - i * Ls;
    const FD f = {Ls, Vh, 1};
    cx<float> yv[12], ev[12];
    ld_spinor<P32>(y, f, 0, s, i, yv);
    ld_spinor<P32>(e, f, 0, s, i, ev);
    const float inv = (float)(1.0 / *enorm);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const cx<float> d = yv[q] - ev[q];
      d2 += (double)d.r * d.r + (double)d.i * d.i;
      yv[q] = inv * d;
    }
    st_spinor<P32>(g, f, 0, s, i, yv);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2 += __shfl_xor(d2, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tsum = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w];
    partial[blockIdx.x] = tsum;
  }
}

// Adam on FP32 master weights; gradient = 2 dL/dW* / batch for (Re, Im)
__global__ void net_adam_kernel(int n, float* w, float* m, float* v, const double* gw, double scale, float lr,
                                float b1, float b2, float eps, float bc1, float bc2, unsigned short* wb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float g = (float)(2.0 * gw[k] * scale);
  const float mk = b1 * m[k] + (1.f - b1) * g;
  const float vk = b2 * v[k] + (1.f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float wk = w[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  w[k] = wk;
  wb[k] = f32_to_bf16(wk);
}

__global__ void net_to_bf16_kernel(int n, const float* w, unsigned short* wb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) wb[k] = f32_to_bf16(w[k]);
}

// complex FP64 BLAS on packed half-fields (one right-hand side)
__global__ void __launch_bounds__(256) cdot_kernel(int n, const double2* a, const double2* b, double* partial) {
  double re = 0.0, im = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double2 x = a[k], y = b[k];  // conj(x) y
    re += x.x * y.x + x.y * y.y;
    im += x.x * y.y - x.y * y.x;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double red[4][2];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = re;
    red[threadIdx.x >> 6][1] = im;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double tsum = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w][threadIdx.x];
    partial[blockIdx.x * 2 + threadIdx.x] = tsum;
  }
}

__global__ void partial_sum2_kernel(const double* partial, int nblk, double* out) {
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b * 2 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// y = y + alpha x  (alpha complex)
__global__ void caxpy_kernel(int n, double ar, double ai, const double2* x, double2* y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double2 a = x[k];
  double2 b = y[k];
  b.x += ar * a.x - ai * a.y;
  b.y += ar * a.y + ai * a.x;
  y[k] = b;
}

// p = z + beta p  (beta complex)
__global__ void cxpby_kernel(int n, const double2* z, double br, double bi, double2* p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double2 a = p[k], zz = z[k];
  p[k] = make_double2(zz.x + br * a.x - bi * a.y, zz.y + br * a.y + bi * a.x);
}

// e_k = x* - x_k for stored FP32 iterates
__global__ void sub_from_kernel(size_t n, const float* xs, float* e) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) e[k] = xs[k] - e[k];
}

// out = sign * num / den (num complex, den real); bad = 1 if den is not a
// positive finite number or the quotient is not finite
__global__ void fgcg_ratio_kernel(const double* num, const double* den, double sign, double* out, int* bad) {
  if (threadIdx.x != 0) return;
  const double d = *den;
  const double re = sign * num[0] / d, im = sign * num[1] / d;
  if (!(d > 0.0) || !isfinite(d) || !isfinite(re) || !isfinite(im)) {
    *bad = 1;
    out[0] = out[1] = 0.0;
    return;
  }
  out[0] = re;
  out[1] = im;
}

// p = z + beta p  (beta complex, on the device)
__global__ void cxpby_dev_kernel(int n, const double2* z, const double* beta, double2* p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double br = beta[0], bi = beta[1];
  const double2 a = p[k], zz = z[k];
  p[k] = make_double2(zz.x + br * a.x - bi * a.y, zz.y + br * a.y + bi * a.x);
}

// y += alpha x  (alpha complex, on the device)
__global__ void caxpy_dev_kernel(int n, const double* alpha, const double2* x, double2* y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double ar = alpha[0], ai = alpha[1];
  const double2 a = x[k];
  double2 b = y[k];
  b.x += ar * a.x - ai * a.y;
  b.y += ar * a.y + ai * a.x;
  y[k] = b;
}

// x += alpha p, r -= alpha q, s -= alpha w; partial |r|^2 and |s|^2 per block
__global__ void __launch_bounds__(256) fgcg_update_kernel(int n, const double* alpha, double2* x, double2* r,
                                                          double2* s, const double2* p, const double2* q,
                                                          const double2* w, double* partial) {
  const double ar = alpha[0], ai = alpha[1];
  double nr = 0.0, ns = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double2 pk = p[k], qk = q[k], wk = w[k];
    double2 xk = x[k], rk = r[k], sk = s[k];
    xk.x += ar * pk.x - ai * pk.y;
    xk.y += ar * pk.y + ai * pk.x;
    rk.x -= ar * qk.x - ai * qk.y;
    rk.y -= ar * qk.y + ai * qk.x;
    sk.x -= ar * wk.x - ai * wk.y;
    sk.y -= ar * wk.y + ai * wk.x;
    x[k] = xk;
    r[k] = rk;
    s[k] = sk;
    nr += rk.x * rk.x + rk.y * rk.y;
    ns += sk.x * sk.x + sk.y * sk.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nr += __shfl_xor(nr, off, 64);
    ns += __shfl_xor(ns, off, 64);
  }
  __shared__ double red[4][2];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = nr;
    red[threadIdx.x >> 6][1] = ns;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double tsum = 0.0;
    for (int wv = 0; wv < (int)(blockDim.x + 63) / 64; ++wv) tsum += red[wv][threadIdx.x];
    partial[threadIdx.x * gridDim.x + blockIdx.x] = tsum;  // [2][nblk]
  }
}

// ---------------------------------------------------------------------------

void launch_pt_layer(const NetLayerArgs& a, bool adj, hipStream_t st) {
  dim3 grid((a.Vh * a.Ls + 255) / 256, (a.Cout + NET_CB - 1) / NET_CB);
  if (adj)
    hipLaunchKernelGGL(pt_layer_kernel<true>, grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(pt_layer_kernel<false>, grid, dim3(256), 0, st, a);
}

void launch_pt_wgrad(const NetGradArgs& a, int nblk, int accumulate, double* gw, hipStream_t st) {
  dim3 grid(nblk, 9 * ((a.Cout + NET_CB - 1) / NET_CB), 2);
  hipLaunchKernelGGL(pt_wgrad_kernel, grid, dim3(256), 0, st, a);
  const int n = 9 * a.Cout * a.Cin * 2;
  hipLaunchKernelGGL(pt_wgrad_final, dim3((n + 255) / 256), dim3(256), 0, st, a.partial, a.Cin, a.Cout, nblk,
                     accumulate, gw);
}

int launch_net_loss(int Vh, int Ls, const float* y, const float* e, float* g, const double* enorm, double* partial,
                    hipStream_t st) {
  const int nblk = (Vh * Ls + 255) / 256;
  hipLaunchKernelGGL(net_loss_kernel, dim3(nblk), dim3(256), 0, st, Vh, Ls, y, e, g, enorm, partial);
  return nblk;
}

void launch_net_adam(int n, float* w, float* m, float* v, const double* gw, double scale, float lr, float b1,
                     float b2, float eps, int step, unsigned short* wb, hipStream_t st) {
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(net_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, w, m, v, gw, scale, lr, b1, b2,
                     eps, bc1, bc2, wb);
}

void launch_net_to_bf16(int n, const float* w, unsigned short* wb, hipStream_t st) {
  hipLaunchKernelGGL(net_to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, w, wb);
}

void launch_cdot(int n, const void* a, const void* b, double* partial, double* out, hipStream_t st) {
  const int nblk = 512;
  hipLaunchKernelGGL(cdot_kernel, dim3(nblk), dim3(256), 0, st, n, (const double2*)a, (const double2*)b, partial);
  hipLaunchKernelGGL(partial_sum2_kernel, dim3(1), dim3(64), 0, st, partial, nblk, out);
}

void launch_caxpy(int n, double ar, double ai, const void* x, void* y, hipStream_t st) {
  hipLaunchKernelGGL(caxpy_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, ar, ai, (const double2*)x,
                     (double2*)y);
}

void launch_cxpby(int n, const void* z, double br, double bi, void* p, hipStream_t st) {
  hipLaunchKernelGGL(cxpby_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, (const double2*)z, br, bi,
                     (double2*)p);
}

void launch_sub_from(size_t n, const float* xs, float* e, hipStream_t st) {
  hipLaunchKernelGGL(sub_from_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, xs, e);
}

void launch_fgcg_ratio(const double* num, const double* den, double sign, double* out, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(fgcg_ratio_kernel, dim3(1), dim3(64), 0, st, num, den, sign, out, bad);
}

void launch_cxpby_dev(int n, const void* z, const double* beta, void* p, hipStream_t st) {
  hipLaunchKernelGGL(cxpby_dev_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, (const double2*)z, beta,
                     (double2*)p);
}

void launch_caxpy_dev(int n, const double* alpha, const void* x, void* y, hipStream_t st) {
  hipLaunchKernelGGL(caxpy_dev_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, alpha, (const double2*)x,
                     (double2*)y);
}

int launch_fgcg_update(int n, const double* alpha, void* x, void* r, void* s, const void* p, const void* q,
                       const void* w, double* partial, hipStream_t st) {
  const int nblk = std::min(1024, (n + 255) / 256);
  hipLaunchKernelGGL(fgcg_update_kernel, dim3(nblk), dim3(256), 0, st, n, alpha, (double2*)x, (double2*)r,
                     (double2*)s, (const double2*)p, (const double2*)q, (const double2*)w, partial);
  return nblk;
}

}  // namespace eofa
