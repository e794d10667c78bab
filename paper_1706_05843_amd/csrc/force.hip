// Link derivative of the hopping term and the EOFA pseudofermion force
// (Sec. IV C, eqn eofa_force).
//
// For 5D fields a, b and one link (x, mu), the derivative of
// a^dag Dhop b along U_mu(x) -> e^{s T} U_mu(x) at s = 0 is, for every
// traceless anti-Hermitian T (Dhop: overall -1/2, eqn Ddwf),
//   -1/2 sum_s [ a^dag(x,s) (1 - g_mu) T U b(x+mu,s) - a^dag(x+mu,s) (1 + g_mu) U^dag T b(x,s) ]
//   = Tr(T y),   y = -1/2 U B1 + 1/2 B2 U^dag,
//   B1 = sum_s Tr_spin[(1 - g_mu) b(x+mu,s) a(x,s)^dag],
//   B2 = sum_s Tr_spin[(1 + g_mu) b(x,s) a(x+mu,s)^dag]
// (U with the boundary phase of the link). In the chiral basis
// g_mu = [[0, A], [A^dag, 0]], so Tr_spin[(1 + sg g_mu) v w^dag] is the sum over
// the two components of h_v h_w^dag with h = up + sg A lo: only projected
// 2-spinors enter.
//
// Layouts: fields canonical complex128 [Ls][T][Z][Y][X][4][3]; links the
// packed FP64 per-parity tables (forward direction mu of site i of parity p
// at ((i * 8 + mu) * 9), phase included); y and the force canonical
// complex128 [4][T][Z][Y][X][3][3].
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "force_internal.h"

namespace eofa {

namespace {

__device__ __forceinline__ void coords_of(const int L[4], int parity, int i, int x[4]) {
  const int hx = L[0] / 2;
  int rest = i / hx;
  const int xh = i - rest * hx;
  x[1] = rest % L[1];
  rest /= L[1];
  x[2] = rest % L[2];
  x[3] = rest / L[2];
  x[0] = 2 * xh + ((parity + x[1] + x[2] + x[3]) & 1);
}

__device__ __forceinline__ size_t lex_of(const int L[4], const int x[4]) {
  return (((size_t)x[3] * L[2] + x[2]) * L[1] + x[1]) * L[0] + x[0];
}

// h = up + sg A lo for the 2 x 3 projected components of a 4 x 3 spinor
// (A = -i sigma_1, -i sigma_2, -i sigma_3, 1 for mu = 0..3)
__device__ __forceinline__ void project(const cx<double>* v, int mu, double sg, cx<double>* h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<double> u0 = v[c], u1 = v[3 + c], l0 = v[6 + c], l1 = v[9 + c];
    if (mu == 0) {
      h[c] = u0 - sg * mul_i(l1);
      h[3 + c] = u1 - sg * mul_i(l0);
    } else if (mu == 1) {
      h[c] = u0 - sg * l1;
      h[3 + c] = u1 + sg * l0;
    } else if (mu == 2) {
      h[c] = u0 - sg * mul_i(l0);
      h[3 + c] = u1 + sg * mul_i(l1);
    } else {
      h[c] = u0 + sg * l0;
      h[3 + c] = u1 + sg * l1;
    }
  }
}

// 12 complex of field f at (s, lex); g5r5: read (gamma_5 R5 f)(s) = gamma_5 f(Ls-1-s)
__device__ __forceinline__ void load12(const double2* f, int Ls, size_t V, int s, size_t lx, bool g5r5,
                                       cx<double>* v) {
  const int ss = g5r5 ? Ls - 1 - s : s;
  const double2* p = f + ((size_t)ss * V + lx) * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 t = p[c];
    const double sgn = (g5r5 && c >= 6) ? -1.0 : 1.0;
    v[c] = {sgn * t.x, sgn * t.y};
  }
}

// B += sum over the two projected components of h_v h_w^dag (3 x 3)
__device__ __forceinline__ void outer_acc(const cx<double>* hv, const cx<double>* hw, cx<double>* B) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> t = B[i * 3 + j];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const cx<double> v = hv[c * 3 + i], w = hw[c * 3 + j];
        t.r += v.r * w.r + v.i * w.i;  // v conj(w)
        t.i += v.i * w.r - v.r * w.i;
      }
      B[i * 3 + j] = t;
    }
}

__global__ void __launch_bounds__(128) dhop_deriv_kernel(DerivArgs d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y, p = blockIdx.z;
  if (i >= d.Vh) return;
  int x[4], xp[4];
  coords_of(d.L, p, i, x);
  for (int k = 0; k < 4; ++k) xp[k] = x[k];
  xp[mu] = (x[mu] + 1) % d.L[mu];
  const size_t V = (size_t)d.L[0] * d.L[1] * d.L[2] * d.L[3];
  const size_t lx = lex_of(d.L, x), lxp = lex_of(d.L, xp);
  const double2* Up = d.links[p] + ((size_t)i * 8 + mu) * 9;
  cx<double> U[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) U[k] = {Up[k].x, Up[k].y};
  cx<double> B1[9], B2[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) B1[k] = B2[k] = {0.0, 0.0};
  for (int s = 0; s < d.Ls; ++s) {
    cx<double> v[12], w[12], hv[6], hw[6];
    // B1: (1 - g_mu) b(x+mu) a(x)^dag
    load12(d.b, d.Ls, V, s, lxp, false, v);
    load12(d.a, d.Ls, V, s, lx, d.g5r5_a, w);
    project(v, mu, -1.0, hv);
    project(w, mu, -1.0, hw);
    outer_acc(hv, hw, B1);
    // B2: (1 + g_mu) b(x) a(x+mu)^dag
    load12(d.b, d.Ls, V, s, lx, false, v);
    load12(d.a, d.Ls, V, s, lxp, d.g5r5_a, w);
    project(v, mu, 1.0, hv);
    project(w, mu, 1.0, hw);
    outer_acc(hv, hw, B2);
  }
  // y = coef (-1/2 U B1 + 1/2 B2 U^dag)
  double2* out = d.y + ((size_t)mu * V + lx) * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<double> t1 = {0.0, 0.0}, t2 = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        t1 = cfma(U[r * 3 + k], B1[k * 3 + c], t1);
        const cx<double> ud = {U[c * 3 + k].r, -U[c * 3 + k].i};  // (U^dag)[k][c]
        t2 = cfma(B2[r * 3 + k], ud, t2);
      }
      const cx<double> yv = {d.coef * 0.5 * (t2.r - t1.r), d.coef * 0.5 * (t2.i - t1.i)};
      double2 o = d.accumulate ? out[r * 3 + c] : make_double2(0.0, 0.0);
      o.x += yv.r;
      o.y += yv.i;
      out[r * 3 + c] = o;
    }
}

// F = sum_a T^a Re Tr(T^a Y) = -1/4 [(Y - Y^dag) - 1/3 Tr(Y - Y^dag)] for the
// basis T^a = i lambda^a / 2 (Tr T^a T^b = -1/2 delta^ab), in place
__global__ void force_project_kernel(size_t nlinks, double2* y) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nlinks) return;
  double2* m = y + k * 9;
  cx<double> Z[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 a = m[r * 3 + c], b = m[c * 3 + r];
      Z[r * 3 + c] = {a.x - b.x, a.y + b.y};  // Y - Y^dag
    }
  const double tr_i = (Z[0].i + Z[4].i + Z[8].i) / 3.0;  // the trace of Y - Y^dag is imaginary
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cx<double> z = Z[r * 3 + c];
      if (r == c) z.i -= tr_i;
      m[r * 3 + c] = make_double2(-0.25 * z.r, -0.25 * z.i);
    }
}

// G-parity in x on the x-doubled lattice: U2(x') = U(x') for x' < Lx,
// conj(U(x' - Lx)) for Lx <= x' < 2 Lx (the flavour-1 copy)
__global__ void double_gauge_kernel(int Lx, size_t rows, const double2* U, double2* U2) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // over 4 * rows * 2Lx sites
  const size_t nsite = (size_t)4 * rows * 2 * Lx;
  if (k >= nsite) return;
  const int xd = (int)(k % (2 * Lx));
  const size_t row = k / (2 * Lx);  // (mu, t, z, y)
  const bool flv = xd >= Lx;
  const double2* src = U + (row * Lx + (flv ? xd - Lx : xd)) * 9;
  double2* dst = U2 + k * 9;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const double2 v = src[c];
    dst[c] = make_double2(v.x, flv ? -v.y : v.y);
  }
}

// physical force F(x) = F2(x) + conj(F2(x + Lx)) from the doubled-lattice one
__global__ void fold_force_kernel(int Lx, size_t rows, const double2* F2, double2* F) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // over 4 * rows * Lx links
  if (k >= (size_t)4 * rows * Lx) return;
  const int x = (int)(k % Lx);
  const size_t row = k / Lx;
  const double2* a = F2 + (row * 2 * Lx + x) * 9;
  const double2* b = F2 + (row * 2 * Lx + x + Lx) * 9;
#pragma unroll
  for (int c = 0; c < 9; ++c) F[k * 9 + c] = make_double2(a[c].x + b[c].x, a[c].y - b[c].y);
}

}  // namespace

void launch_double_gauge(int Lx, size_t rows, const void* U, void* U2, hipStream_t st) {
  const size_t n = (size_t)4 * rows * 2 * Lx;
  hipLaunchKernelGGL(double_gauge_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Lx, rows,
                     (const double2*)U, (double2*)U2);
}

void launch_fold_force(int Lx, size_t rows, const void* F2, void* F, hipStream_t st) {
  const size_t n = (size_t)4 * rows * Lx;
  hipLaunchKernelGGL(fold_force_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Lx, rows,
                     (const double2*)F2, (double2*)F);
}

void launch_dhop_deriv(const DerivArgs& d, hipStream_t st) {
  dim3 grid((d.Vh + 127) / 128, 4, 2);
  hipLaunchKernelGGL(dhop_deriv_kernel, grid, dim3(128), 0, st, d);
}

void launch_force_project(size_t nlinks, void* y, hipStream_t st) {
  hipLaunchKernelGGL(force_project_kernel, dim3((unsigned)((nlinks + 255) / 256)), dim3(256), 0, st, nlinks,
                     (double2*)y);
}

}  // namespace eofa
