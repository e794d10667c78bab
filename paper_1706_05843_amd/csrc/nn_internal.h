// Internal interface of the parallel-transport network kernels (nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace eofa {

constexpr int NET_MAXC = 8;       // most channels per layer
constexpr int NET_TERMS = 20;     // stencil terms per channel pair
constexpr int NET_DOT_BLOCKS = 256;  // work-groups of the residual-loss reductions

struct NetLayerArgs {
  const float* xin[2];       // packed FP32 activations of both parities, Cin channels
  float* yout;               // packed FP32 output of parity `parity`, Cout channels
  const unsigned short* w;   // bfloat16 (re, im) [20][Cout_fwd][Cin_fwd] of the forward layer
  const float* links;        // FP32 links of the output parity [Vh][8][9] complex
  const int* nbr;            // [Vh][8] neighbour index in the other parity
  int Vh, Ls, Cin, Cout;     // of this (forward or adjoint) application
  int parity;
};

struct NetGradArgs {
  const float* x[2];         // layer input, both parities, Cin channels
  const float* g[2];         // dL/dy* at the layer output, both parities, Cout channels
  const float* links[2];
  const int* nbr[2];
  double* partial;           // [20*Cin][2][Cout][nblk][2]
  int Vh, Ls, Cin, Cout;
};

void launch_pt_layer(const NetLayerArgs& a, bool adj, hipStream_t st);
void launch_pt_wgrad(const NetGradArgs& a, int nblk, int accumulate, double* gw, hipStream_t st);
// residual loss of one pair: partial [3 * NET_DOT_BLOCKS] scratch; *loss =
// 1 - |<a, r>|^2/(|a|^2 |r|^2) (rnorm = |r|^2 on the device), coef[3] the
// coefficients of dL/da*, out = dL/da* (one-channel FP32 odd half-fields)
void launch_net_resid(int Vh, int Ls, const float* av, const float* rv, const double* rnorm, double* partial,
                      double* loss, double* coef, float* out, hipStream_t st);
int launch_net_loss(int Vh, int Ls, const float* y, const float* e, float* g, const double* enorm, double* partial,
                    hipStream_t st);
void launch_net_adam(int n, float* w, float* m, float* v, const double* gw, double scale, float lr, float b1,
                     float b2, float eps, int step, unsigned short* wb, hipStream_t st);
void launch_net_to_bf16(int n, const float* w, unsigned short* wb, hipStream_t st);
void launch_cdot(int n, const void* a, const void* b, double* partial, double* out, hipStream_t st);
void launch_caxpy(int n, double ar, double ai, const void* x, void* y, hipStream_t st);
void launch_cxpby(int n, const void* z, double br, double bi, void* p, hipStream_t st);
void launch_sub_from(size_t n, const float* xs, float* e, hipStream_t st);
void launch_fgcg_ratio(const double* num, const double* den, double sign, double* out, int* bad, hipStream_t st);
void launch_cxpby_dev(int n, const void* z, const double* beta, void* p, hipStream_t st);
// flexible CG window: up to FG_CHUNK previous directions per pass
constexpr int FG_CHUNK = 8;
struct FgPtrs {
  const void* v[FG_CHUNK];     // packed FP64 odd half-fields (q_j or p_j)
  const double* ww[FG_CHUNK];  // <p_j, A p_j> on the device (coefficients only)
};
// beta_j = -<q_j, z>/ww_j for j < nq into beta[2 nq] (partial: 2 * 512 * nq
// doubles of scratch); bad = 1 on a non-positive or non-finite ww_j or beta_j
void launch_fgcg_orth_coefs(int n, int nq, const FgPtrs& q, const void* z, double* partial, double* beta, int* bad,
                            hipStream_t st);
// p += sum_j beta_j p_j
void launch_caxpy_multi(int n, int nq, const FgPtrs& pp, const double* beta, void* p, hipStream_t st);
void launch_caxpy_dev(int n, const double* alpha, const void* x, void* y, hipStream_t st);
// returns the number of blocks; partial holds [2][nblk] (|r|^2 then |s|^2)
int launch_fgcg_update(int n, const double* alpha, void* x, void* r, void* s, const void* p, const void* q,
                       const void* w, double* partial, hipStream_t st);

}  // namespace eofa
