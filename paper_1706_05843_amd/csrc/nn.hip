// Kernels of the gauge-covariant parallel-transport network (flexible
// preconditioner) and of flexible CG. Not part of the paper's method: the
// layer form, losses and optimiser are this library's choices.
//
// Layer C_in -> C_out, output parity p, 20 terms per channel pair:
//   y_c(x, s) = sum_t sum_c' W[t][c][c'] (S_t X_c')(x, s),
//   S_0 = P_+, S_1 = P_-, S_{2+e} = T_e, S_{10+e} = g_mu(e) T_e (e = 0..7),
//   S_18 X(s) = P_+ X(s-1), S_19 X(s) = P_- X(s+1) (cyclic in s),
// with the eight transports T_e of the hop kernels' per-parity links
// (e < 4: U_mu(x) X(x+mu), mu = e; e >= 4: U_mu(x-mu)^dag X(x-mu), mu = e-4;
// boundary phases included). Activations are packed FP32 half-fields with
// the channel as the right-hand-side index. Weights: bfloat16 pairs
// (re, im) [20][C_out][C_in], FP32 arithmetic.
// Adjoint in X: conj(W[t'][c'][c]) S_t'^dag with T_e^dag = T_{e^4}, g_mu
// Hermitian and commuting with the transports, P_+- Hermitian and the s
// shifts reversed.
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

__device__ __forceinline__ cx<float> times_i(cx<float> a) { return {-a.i, a.r}; }

// one chirality half of a packed FP32 spinor: h = 0 the P_+ components
// 0..5 (into v[0..5]), h = 1 the P_- components 6..11 (into v[6..11])
__device__ __forceinline__ void ld_half32(const float* base, const FD& f, int r, int s, int i, int h,
                                          cx<float>* v) {
  const size_t e0 = eidx(f, r, 0, s, i), qs = qstride(f);
#pragma unroll
  for (int q = 0; q < 3; ++q) ld_pair<P32>(base, e0 + (3 * h + q) * qs, v[6 * h + 2 * q], v[6 * h + 2 * q + 1]);
}

// g = g_mu v in the chiral basis of the field layout:
// g_mu = [[0, A_mu], [A_mu^dag, 0]], A = -i sigma_1, -i sigma_2, -i sigma_3, 1
__device__ __forceinline__ void gamma_mul(int mu, const cx<float>* v, cx<float>* g) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<float> u0 = v[c], u1 = v[3 + c], l0 = v[6 + c], l1 = v[9 + c];
    if (mu == 0) {
      g[c] = -1.f * times_i(l1);
      g[3 + c] = -1.f * times_i(l0);
      g[6 + c] = times_i(u1);
      g[9 + c] = times_i(u0);
    } else if (mu == 1) {
      g[c] = -1.f * l1;
      g[3 + c] = l0;
      g[6 + c] = u1;
      g[9 + c] = -1.f * u0;
    } else if (mu == 2) {
      g[c] = -1.f * times_i(l0);
      g[3 + c] = times_i(l1);
      g[6 + c] = times_i(u0);
      g[9 + c] = -1.f * times_i(u1);
    } else {
      g[c] = l0;
      g[3 + c] = l1;
      g[6 + c] = u0;
      g[9 + c] = u1;
    }
  }
}

// weight of term t from input channel ci to output channel c of this
// application; the adjoint reads conj(W[t][ci][c]) of the forward layer
// (whose C_out is this application's C_in)
template <bool ADJ>
__device__ __forceinline__ cx<float> wload(const NetLayerArgs& a, int t, int c, int ci) {
  const size_t k = ADJ ? (((size_t)t * a.Cin + ci) * a.Cout + c) * 2 : (((size_t)t * a.Cout + c) * a.Cin + ci) * 2;
  const float wr = bf16_to_f32(a.w[k]), wi = bf16_to_f32(a.w[k + 1]);
  return {wr, ADJ ? -wi : wi};
}

// One thread: one 5D site (i, s) of the output parity and a block of CB
// output channels c0 .. c0+CB-1. The work-group first stages the weights it
// needs, W[t][c0+cc][ci] as FP32 complex (conjugated and transposed for the
// adjoint), in LDS: every lane reads the same weight, which LDS broadcasts.
// Per transport direction e the term pair W[2+e] + W[10+e] g_mu is applied
// in one of two orders (g_mu commutes with the link):
//  * TF (transport first): each input channel is transported once and then
//    mixed into the CB outputs: C_in link products, accumulators only;
//  * otherwise mix first: z_c = sum_c' (W[2+e] + W[10+e] g_mu) X_c'(neighbour)
//    for the CB outputs, then one link product per output: CB link products,
//    but CB more spinors of registers.
// The launcher takes TF when C_in <= CB. Registers: 48 CB (accumulators),
// plus 48 CB for mix first.
template <bool ADJ, int CB, bool TF>
__global__ void __launch_bounds__(256) pt_layer_kernel(NetLayerArgs a) {
  __shared__ float2 s_w[NET_TERMS * 4 * NET_MAXC];  // [t][cc][ci], CB <= 4
  const int c0 = blockIdx.y * CB;
  const int nco = min(CB, a.Cout - c0);
  for (int k = threadIdx.x; k < NET_TERMS * CB * a.Cin; k += blockDim.x) {
    const int ci = k % a.Cin, cc = (k / a.Cin) % CB, t = k / (a.Cin * CB);
    float2 w = {0.f, 0.f};
    if (cc < nco) {
      const cx<float> v = wload<ADJ>(a, t, c0 + cc, ci);
      w = {v.r, v.i};
    }
    s_w[k] = w;
  }
  __syncthreads();
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.Vh * a.Ls) return;
  auto W = [&](int t, int cc, int ci) {
    const float2 w = s_w[(t * CB + cc) * a.Cin + ci];
    return cx<float>{w.x, w.y};
  };
  const int i = idx / a.Ls, s = idx - i * a.Ls;
  const int p = a.parity;
  const FD fin = {a.Ls, a.Vh, a.Cin};
  cx<float> acc[CB][12];
#pragma unroll
  for (int cc = 0; cc < CB; ++cc)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[cc][k] = {0.f, 0.f};
  // same-parity terms: P_+ and P_- at (x, s); P_+ X(s-1) and P_- X(s+1),
  // in the adjoint P_+ X(s+1) and P_- X(s-1)
  {
    const int sm = s == 0 ? a.Ls - 1 : s - 1, sp = s == a.Ls - 1 ? 0 : s + 1;
    const int s_up = ADJ ? sp : sm, s_lo = ADJ ? sm : sp;
    for (int ci = 0; ci < a.Cin; ++ci) {
      cx<float> v[12], xu[12], xl[12];
      ld_spinor<P32>(a.xin[p], fin, ci, s, i, v);
      ld_half32(a.xin[p], fin, ci, s_up, i, 0, xu);
      ld_half32(a.xin[p], fin, ci, s_lo, i, 1, xl);
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        const cx<float> w0 = W(0, cc, ci), w1 = W(1, cc, ci), w18 = W(18, cc, ci), w19 = W(19, cc, ci);
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[cc][q] = cfma(w18, xu[q], cfma(w0, v[q], acc[cc][q]));
#pragma unroll
        for (int q = 6; q < 12; ++q) acc[cc][q] = cfma(w19, xl[q], cfma(w1, v[q], acc[cc][q]));
      }
    }
  }
  for (int e = 0; e < 8; ++e) {
    const int j = a.nbr[(size_t)i * 8 + e];
    const int te = ADJ ? (e ^ 4) : e;  // T_e^dag = T_{e^4}
    const int mu = e & 3;
    const float2* L = (const float2*)a.links + ((size_t)i * 8 + e) * 9;
    if constexpr (TF) {
      for (int ci = 0; ci < a.Cin; ++ci) {
        cx<float> v[12], gv[12];
        ld_spinor<P32>(a.xin[1 - p], fin, ci, s, j, v);
        link_mul(L, v);
        gamma_mul(mu, v, gv);
#pragma unroll
        for (int cc = 0; cc < CB; ++cc) {
          const cx<float> wa = W(2 + te, cc, ci), wb = W(10 + te, cc, ci);
#pragma unroll
          for (int q = 0; q < 12; ++q) acc[cc][q] = cfma(wb, gv[q], cfma(wa, v[q], acc[cc][q]));
        }
      }
    } else {
      cx<float> z[CB][12];
#pragma unroll
      for (int cc = 0; cc < CB; ++cc)
#pragma unroll
        for (int k = 0; k < 12; ++k) z[cc][k] = {0.f, 0.f};
      for (int ci = 0; ci < a.Cin; ++ci) {
        cx<float> v[12], gv[12];
        ld_spinor<P32>(a.xin[1 - p], fin, ci, s, j, v);
        gamma_mul(mu, v, gv);
#pragma unroll
        for (int cc = 0; cc < CB; ++cc) {
          const cx<float> wa = W(2 + te, cc, ci), wb = W(10 + te, cc, ci);
#pragma unroll
          for (int q = 0; q < 12; ++q) z[cc][q] = cfma(wb, gv[q], cfma(wa, v[q], z[cc][q]));
        }
      }
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) {
        if (cc >= nco) break;
        link_mul(L, z[cc]);
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[cc][q] = acc[cc][q] + z[cc][q];
      }
    }
  }
  const FD fo = {a.Ls, a.Vh, a.Cout};
#pragma unroll
  for (int cc = 0; cc < CB; ++cc) {
    if (cc >= nco) break;
    st_spinor<P32>(a.yout, fo, c0 + cc, s, i, acc[cc]);
  }
}

// dL/dW*[t][c][ci] partial sums: sum over sites of G_c(x) . conj((S_t X_ci)(x)).
// Work-group (blk, grp * ncb + cb, parity) computes two terms of group grp:
// grp < 8 the transport e = grp (terms 2+e and 10+e), grp = 8 the same-site
// chirality terms (0, 1), grp = 9 the s shifts (18, 19); output channels
// cb*WG_CB .. +WG_CB-1, all input channels. Each thread loads its site's G_c
// once and each transported input once per channel block.
constexpr int WG_CB = 2;
constexpr int WG_GROUPS = 10;

__global__ void __launch_bounds__(256) pt_wgrad_kernel(NetGradArgs a) {
  const int ncb = (a.Cout + WG_CB - 1) / WG_CB;
  const int grp = blockIdx.y / ncb, cb = blockIdx.y - grp * ncb;
  const int c0 = cb * WG_CB;
  const int nco = min(WG_CB, a.Cout - c0);
  const int p = blockIdx.z;
  const FD fx = {a.Ls, a.Vh, a.Cin}, fg = {a.Ls, a.Vh, a.Cout};
  // [cc][ci][term a / b]
  float ar[WG_CB][NET_MAXC][2], ai[WG_CB][NET_MAXC][2];
#pragma unroll
  for (int cc = 0; cc < WG_CB; ++cc)
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci)
#pragma unroll
      for (int h = 0; h < 2; ++h) ar[cc][ci][h] = ai[cc][ci][h] = 0.f;
  const int n = a.Vh * a.Ls;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    const int i = idx / a.Ls, s = idx - i * a.Ls;
    cx<float> g[WG_CB][12];
#pragma unroll
    for (int cc = 0; cc < WG_CB; ++cc) {
      if (cc >= nco) break;
      ld_spinor<P32>(a.g[p], fg, c0 + cc, s, i, g[cc]);
    }
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci) {
      if (ci >= a.Cin) break;
      // va = S_ta X_ci, vb = S_tb X_ci at (x, s)
      cx<float> va[12], vb[12];
      if (grp < 8) {
        const int j = a.nbr[p][(size_t)i * 8 + grp];
        ld_spinor<P32>(a.x[1 - p], fx, ci, s, j, va);
        link_mul((const float2*)a.links[p] + ((size_t)i * 8 + grp) * 9, va);
        gamma_mul(grp & 3, va, vb);
      } else if (grp == 8) {
        ld_spinor<P32>(a.x[p], fx, ci, s, i, va);
#pragma unroll
        for (int q = 0; q < 12; ++q) vb[q] = va[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) vb[q] = {0.f, 0.f};
#pragma unroll
        for (int q = 6; q < 12; ++q) va[q] = {0.f, 0.f};
      } else {
        ld_half32(a.x[p], fx, ci, s == 0 ? a.Ls - 1 : s - 1, i, 0, va);
        ld_half32(a.x[p], fx, ci, s == a.Ls - 1 ? 0 : s + 1, i, 1, vb);
#pragma unroll
        for (int q = 0; q < 6; ++q) vb[q] = {0.f, 0.f};
#pragma unroll
        for (int q = 6; q < 12; ++q) va[q] = {0.f, 0.f};
      }
#pragma unroll
      for (int cc = 0; cc < WG_CB; ++cc) {
        if (cc >= nco) break;
        float sr0 = 0.f, si0 = 0.f, sr1 = 0.f, si1 = 0.f;
#pragma unroll
        for (int q = 0; q < 12; ++q) {  // g * conj(v)
          sr0 = fmaf(g[cc][q].r, va[q].r, fmaf(g[cc][q].i, va[q].i, sr0));
          si0 = fmaf(g[cc][q].i, va[q].r, fmaf(-g[cc][q].r, va[q].i, si0));
          sr1 = fmaf(g[cc][q].r, vb[q].r, fmaf(g[cc][q].i, vb[q].i, sr1));
          si1 = fmaf(g[cc][q].i, vb[q].r, fmaf(-g[cc][q].r, vb[q].i, si1));
        }
        ar[cc][ci][0] += sr0;
        ai[cc][ci][0] += si0;
        ar[cc][ci][1] += sr1;
        ai[cc][ci][1] += si1;
      }
    }
  }
  // reduce the WG_CB x C_in x 2 complex sums over the work-group
  constexpr int NV = 2 * WG_CB * NET_MAXC * 2;  // (cc, ci, h, comp)
  __shared__ double red[4][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int cc = 0; cc < WG_CB; ++cc)
#pragma unroll
    for (int ci = 0; ci < NET_MAXC; ++ci)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (cc >= nco || ci >= a.Cin) continue;
        double vr = ar[cc][ci][h], vi = ai[cc][ci][h];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          vr += __shfl_xor(vr, off, 64);
          vi += __shfl_xor(vi, off, 64);
        }
        if (lane == 0) {
          const int k = ((cc * NET_MAXC + ci) * 2 + h) * 2;
          red[wv][k] = vr;
          red[wv][k + 1] = vi;
        }
      }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < NV) {
    const int comp = k & 1, h = (k >> 1) & 1, ci = (k >> 2) % NET_MAXC, cc = (k >> 2) / NET_MAXC;
    if (cc < nco && ci < a.Cin) {
      double tsum = 0.0;
      for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w][k];
      const int t = grp < 8 ? (h ? 10 + grp : 2 + grp) : grp == 8 ? h : 18 + h;
      const int y = t * a.Cin + ci, c = c0 + cc;
      a.partial[((((size_t)y * 2 + p) * a.Cout + c) * gridDim.x + blockIdx.x) * 2 + comp] = tsum;
    }
  }
}

// gW[t][c][ci] (+)= sum over parity and blocks (fixed order), as (re, im) doubles
__global__ void pt_wgrad_final(const double* partial, int Cin, int Cout, int nblk, int accumulate, double* gw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // over NET_TERMS*Cout*Cin*2
  if (k >= NET_TERMS * Cout * Cin * 2) return;
  const int comp = k & 1, rest = k >> 1;
  const int ci = rest % Cin, c = (rest / Cin) % Cout, t = rest / (Cin * Cout);
  const int y = t * Cin + ci;
  double s = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int b = 0; b < nblk; ++b) s += partial[((((size_t)y * 2 + p) * Cout + c) * nblk + b) * 2 + comp];
  gw[k] = accumulate ? gw[k] + s : s;
}

// residual loss: partial sums of <a, r> (re, im) and |a|^2 over one-channel
// FP32 odd half-fields, as [3][nblk]
__global__ void __launch_bounds__(256) net_dot_kernel(int Vh, int Ls, const float* av, const float* rv,
                                                      double* partial) {
  const FD f = {Ls, Vh, 1};
  double cr = 0.0, ci = 0.0, na = 0.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < Vh * Ls; idx += gridDim.x * blockDim.x) {
    const int i = idx / Ls, s = idx - i * Ls;
    cx<float> x[12], y[12];
    ld_spinor<P32>(av, f, 0, s, i, x);
    ld_spinor<P32>(rv, f, 0, s, i, y);
#pragma unroll
    for (int q = 0; q < 12; ++q) {  // conj(a) r
      cr += (double)x[q].r * y[q].r + (double)x[q].i * y[q].i;
      ci += (double)x[q].r * y[q].i - (double)x[q].i * y[q].r;
      na += (double)x[q].r * x[q].r + (double)x[q].i * x[q].i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cr += __shfl_xor(cr, off, 64);
    ci += __shfl_xor(ci, off, 64);
    na += __shfl_xor(na, off, 64);
  }
  __shared__ double red[4][3];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = cr;
    red[threadIdx.x >> 6][1] = ci;
    red[threadIdx.x >> 6][2] = na;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double tsum = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w][threadIdx.x];
    partial[threadIdx.x * gridDim.x + blockIdx.x] = tsum;
  }
}

// loss = 1 - |c|^2/(|a|^2 |r|^2), c = <a, r>, and the coefficients of
// dL/da* = alpha a + beta r: alpha = |c|^2/(|a|^4 |r|^2), beta = -conj(c)/(|a|^2 |r|^2)
// as coef = (alpha, Re beta, Im beta); a = 0 (or a non-finite sum) gives
// loss 1 and zero coefficients
__global__ void net_resid_coef_kernel(const double* partial, int nblk, const double* rnorm, double* loss,
                                      double* coef) {
  if (threadIdx.x != 0) return;
  double cr = 0.0, ci = 0.0, na = 0.0;
  for (int b = 0; b < nblk; ++b) {
    cr += partial[b];
    ci += partial[nblk + b];
    na += partial[2 * nblk + b];
  }
  const double nr = *rnorm, c2 = cr * cr + ci * ci;
  const double l = 1.0 - c2 / (na * nr);
  if (!(na > 0.0) || !(nr > 0.0) || !isfinite(l)) {
    *loss = 1.0;
    coef[0] = coef[1] = coef[2] = 0.0;
    return;
  }
  *loss = l;
  coef[0] = c2 / (na * na * nr);
  coef[1] = -cr / (na * nr);
  coef[2] = ci / (na * nr);
}

// out = alpha a + beta r (one-channel FP32 odd half-fields)
__global__ void __launch_bounds__(256) net_combine_kernel(int Vh, int Ls, const float* av, const float* rv,
                                                          const double* coef, float* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Vh * Ls) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, 1};
  const float al = (float)coef[0];
  const cx<float> be = {(float)coef[1], (float)coef[2]};
  cx<float> x[12], y[12];
  ld_spinor<P32>(av, f, 0, s, i, x);
  ld_spinor<P32>(rv, f, 0, s, i, y);
#pragma unroll
  for (int q = 0; q < 12; ++q) x[q] = cfma(be, y[q], al * x[q]);
  st_spinor<P32>(out, f, 0, s, i, x);
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

// sum of nblk (re, im) partials in a fixed order: 128 strided sums per
// component, then a tree (256 threads)
__device__ __forceinline__ void sum_pairs_256(const double* partial, int nblk, double* red) {
  const int c = threadIdx.x & 1;
  double s = 0.0;
  for (int b = threadIdx.x >> 1; b < nblk; b += 128) s += partial[b * 2 + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 2; w >>= 1) {  // w even: t and t + w hold the same component
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) partial_sum2_kernel(const double* partial, int nblk, double* out) {
  __shared__ double red[256];
  sum_pairs_256(partial, nblk, red);
  if (threadIdx.x < 2) out[threadIdx.x] = red[threadIdx.x];
}

// <q_j, z> partial sums for j < nq, as [nq][nblk][2]
__global__ void __launch_bounds__(256) cdot_multi_kernel(int n, int nq, FgPtrs q, const double2* z, double* partial) {
  double re[FG_CHUNK], im[FG_CHUNK];
#pragma unroll
  for (int j = 0; j < FG_CHUNK; ++j) re[j] = im[j] = 0.0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double2 y = z[k];
#pragma unroll
    for (int j = 0; j < FG_CHUNK; ++j) {
      if (j >= nq) break;
      const double2 x = ((const double2*)q.v[j])[k];  // conj(x) y
      re[j] += x.x * y.x + x.y * y.y;
      im[j] += x.x * y.y - x.y * y.x;
    }
  }
  __shared__ double red[4][2 * FG_CHUNK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < FG_CHUNK; ++j) {
    if (j >= nq) break;
    double a = re[j], b = im[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane == 0) {
      red[wv][2 * j] = a;
      red[wv][2 * j + 1] = b;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * nq) {
    double tsum = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) tsum += red[w][threadIdx.x];
    partial[((size_t)(threadIdx.x >> 1) * gridDim.x + blockIdx.x) * 2 + (threadIdx.x & 1)] = tsum;
  }
}

// work-group j: beta_j = -<q_j, z> / ww_j; bad = 1 if ww_j is not a positive
// finite number or beta_j is not finite
__global__ void __launch_bounds__(256) fgcg_coef_kernel(const double* partial, int nblk, FgPtrs q, double* beta,
                                                        int* bad) {
  const int j = blockIdx.x;
  __shared__ double red[256];
  sum_pairs_256(partial + (size_t)j * nblk * 2, nblk, red);
  if (threadIdx.x != 0) return;
  const double d = *q.ww[j];
  const double re = -red[0] / d, im = -red[1] / d;
  if (!(d > 0.0) || !isfinite(d) || !isfinite(re) || !isfinite(im)) {
    *bad = 1;
    beta[2 * j] = beta[2 * j + 1] = 0.0;
    return;
  }
  beta[2 * j] = re;
  beta[2 * j + 1] = im;
}

// p += sum_j beta_j p_j, j in order
__global__ void __launch_bounds__(256) caxpy_multi_kernel(int n, int nq, FgPtrs pp, const double* beta, double2* p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2 acc = p[k];
#pragma unroll
  for (int j = 0; j < FG_CHUNK; ++j) {
    if (j >= nq) break;
    const double br = beta[2 * j], bi = beta[2 * j + 1];
    const double2 a = ((const double2*)pp.v[j])[k];
    acc.x += br * a.x - bi * a.y;
    acc.y += br * a.y + bi * a.x;
  }
  p[k] = acc;
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

template <int CB, bool TF>
void launch_pt_layer_cb(const NetLayerArgs& a, bool adj, hipStream_t st) {
  dim3 grid((a.Vh * a.Ls + 255) / 256, (a.Cout + CB - 1) / CB);
  if (adj)
    hipLaunchKernelGGL((pt_layer_kernel<true, CB, TF>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((pt_layer_kernel<false, CB, TF>), grid, dim3(256), 0, st, a);
}

// channel block and order by shape: one output channel mixes first (one
// link product per direction); few inputs transport first; many inputs and
// outputs mix first in blocks of 2
void launch_pt_layer(const NetLayerArgs& a, bool adj, hipStream_t st) {
  if (a.Cout == 1)
    launch_pt_layer_cb<1, false>(a, adj, st);
  else if (a.Cout == 2 && a.Cin <= 2)
    launch_pt_layer_cb<2, true>(a, adj, st);
  else if (a.Cin <= 4)
    launch_pt_layer_cb<4, true>(a, adj, st);
  else
    launch_pt_layer_cb<2, false>(a, adj, st);
}

void launch_pt_wgrad(const NetGradArgs& a, int nblk, int accumulate, double* gw, hipStream_t st) {
  dim3 grid(nblk, WG_GROUPS * ((a.Cout + WG_CB - 1) / WG_CB), 2);
  hipLaunchKernelGGL(pt_wgrad_kernel, grid, dim3(256), 0, st, a);
  const int n = NET_TERMS * a.Cout * a.Cin * 2;
  hipLaunchKernelGGL(pt_wgrad_final, dim3((n + 255) / 256), dim3(256), 0, st, a.partial, a.Cin, a.Cout, nblk,
                     accumulate, gw);
}

void launch_net_resid(int Vh, int Ls, const float* av, const float* rv, const double* rnorm, double* partial,
                      double* loss, double* coef, float* out, hipStream_t st) {
  const int n = Vh * Ls;
  const int nblk = std::min(NET_DOT_BLOCKS, (n + 255) / 256);
  hipLaunchKernelGGL(net_dot_kernel, dim3(nblk), dim3(256), 0, st, Vh, Ls, av, rv, partial);
  hipLaunchKernelGGL(net_resid_coef_kernel, dim3(1), dim3(64), 0, st, partial, nblk, rnorm, loss, coef);
  hipLaunchKernelGGL(net_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, st, Vh, Ls, av, rv, coef, out);
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
  hipLaunchKernelGGL(partial_sum2_kernel, dim3(1), dim3(256), 0, st, partial, nblk, out);
}

void launch_fgcg_orth_coefs(int n, int nq, const FgPtrs& q, const void* z, double* partial, double* beta, int* bad,
                            hipStream_t st) {
  const int nblk = 512;
  hipLaunchKernelGGL(cdot_multi_kernel, dim3(nblk), dim3(256), 0, st, n, nq, q, (const double2*)z, partial);
  hipLaunchKernelGGL(fgcg_coef_kernel, dim3(nq), dim3(256), 0, st, partial, nblk, q, beta, bad);
}

void launch_caxpy_multi(int n, int nq, const FgPtrs& pp, const double* beta, void* p, hipStream_t st) {
  hipLaunchKernelGGL(caxpy_multi_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, nq, pp, beta, (double2*)p);
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
