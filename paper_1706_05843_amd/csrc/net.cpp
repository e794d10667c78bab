// Gauge-covariant parallel-transport network: object, inference, gradients
// and Adam training (host side; kernels in nn.hip). This part is not in the
// paper: it is the learned flexible preconditioner of this library.
//
// Network N = B^dag B, B = L_{L-1} ... L_0 with channels ch[l] -> ch[l+1],
// ch[0] = ch[L] = 1. Input: an odd-sublattice packed FP32 field (one
// channel), embedded in the full lattice with zero even sites; output: the
// odd part of B^dag B of it. Activations kept for the gradients: X[0..L] of
// B (X[0] the embedded input) and Y[0..L-1] of B^dag (Y[k-1] = L_{k-1}^dag
// Y[k], Y[L] = X[L]). Losses (see eofa_net_loss_grad): the error loss over
// pairs (r, e) and the scale-free residual loss over residuals r;
// gradients are dL/dW* (Wirtinger); Adam steps on (Re W, Im W) with
// 2 dL/dW* / batch, FP32 master weights, bfloat16 weights in the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "nn_internal.h"

using namespace eofa;

struct eofa_net {
  int L = 0;
  std::vector<int> ch;
  std::vector<size_t> woff;  // complex-weight offset of each layer
  size_t nw = 0;             // complex weights in total
  float* w32 = nullptr;      // FP32 master (re, im) [2*nw]
  float* m = nullptr;
  float* v = nullptr;
  unsigned short* wb = nullptr;  // bfloat16 copy used by the kernels
  double* gw = nullptr;          // dL/dW* accumulator (re, im)
  int step = 0;
  // activations: act[l][parity] = X[l] and yact[k][parity] = Y[k] with
  // ch[l] (ch[k]) channels, grad buffers g[2][parity]
  size_t sized_for = 0;  // Vh*Ls the buffers fit
  std::vector<void*> act;
  std::vector<void*> yact;
  void* gbuf[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* zero = nullptr;      // an all-zero one-channel half field
  void* ay = nullptr;        // residual loss: A y (one channel)
  void* dg = nullptr;        // residual loss: dL/d(A y)* (one channel)
  double* coef = nullptr;    // residual loss: the 3 coefficients of dL/d(A y)*
  double* partial = nullptr;
  size_t partial_n = 0;
  double* dev_scalars = nullptr;  // |e|^2 per pair
  size_t dev_scalars_n = 0;
};

namespace {

int nfail(int code, const std::string& m) { return set_error(code, m); }

#define NHIP(call)                                                                                         \
  do {                                                                                                     \
    hipError_t e_ = (call);                                                                                \
    if (e_ != hipSuccess) return nfail(EOFA_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_));    \
  } while (0)
#define NCHK(call)                  \
  do {                              \
    int c_ = (call);                \
    if (c_ != EOFA_OK) return c_;   \
  } while (0)

constexpr int WGRAD_BLOCKS = 256;
// weight-gradient partial sums [20*C_in][2][C_out][WGRAD_BLOCKS][2], then the loss partials
constexpr size_t WGRAD_PARTIAL = (size_t)NET_TERMS * NET_MAXC * 2 * NET_MAXC * WGRAD_BLOCKS * 2;

double* loss_partial(eofa_net* N) { return N->partial + WGRAD_PARTIAL; }

size_t half_bytes(const Geometry& g, int channels) { return packed_bytes(P32, g, channels); }

int dmalloc(void** p, size_t n) {
  if (hipMalloc(p, n) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return nfail(EOFA_ERR_OOM, "hipMalloc failed in the network");
  }
  return EOFA_OK;
}

void free_acts(eofa_net* N) {
  for (auto* v : {&N->act, &N->yact}) {
    for (void* p : *v)
      if (p) (void)hipFree(p);
    v->clear();
  }
  for (auto& a : N->gbuf)
    for (auto& b : a)
      if (b) {
        (void)hipFree(b);
        b = nullptr;
      }
  for (void** b : {&N->zero, &N->ay, &N->dg, (void**)&N->coef})
    if (*b) {
      (void)hipFree(*b);
      *b = nullptr;
    }
  N->sized_for = 0;
}

int ensure_acts(eofa_ctx* C, eofa_net* N, hipStream_t st) {
  const size_t key = (size_t)C->g.Vh * C->g.Ls;
  if (N->sized_for == key) return EOFA_OK;
  free_acts(N);
  int cmax = 1;
  for (int c : N->ch) cmax = std::max(cmax, c);
  N->act.assign(2 * (N->L + 1), nullptr);
  for (int l = 0; l <= N->L; ++l)
    for (int p = 0; p < 2; ++p) NCHK(dmalloc(&N->act[2 * l + p], half_bytes(C->g, N->ch[l])));
  N->yact.assign(2 * N->L, nullptr);
  for (int k = 0; k < N->L; ++k)
    for (int p = 0; p < 2; ++p) NCHK(dmalloc(&N->yact[2 * k + p], half_bytes(C->g, N->ch[k])));
  for (auto& a : N->gbuf)
    for (auto& b : a) NCHK(dmalloc(&b, half_bytes(C->g, cmax)));
  NCHK(dmalloc(&N->zero, half_bytes(C->g, 1)));
  NCHK(dmalloc(&N->ay, half_bytes(C->g, 1)));
  NCHK(dmalloc(&N->dg, half_bytes(C->g, 1)));
  NCHK(dmalloc((void**)&N->coef, 4 * sizeof(double)));
  NHIP(hipMemsetAsync(N->zero, 0, half_bytes(C->g, 1), st));
  const size_t pn = WGRAD_PARTIAL;
  const size_t ln = std::max((size_t)(C->g.Vh * C->g.Ls + 255) / 256, (size_t)3 * NET_DOT_BLOCKS);
  if (N->partial_n < pn + ln) {
    if (N->partial) (void)hipFree(N->partial);
    N->partial_n = pn + ln;
    NCHK(dmalloc((void**)&N->partial, N->partial_n * sizeof(double)));
  }
  N->sized_for = key;
  return EOFA_OK;
}

// Y[k] of B^dag (Y[L] = X[L])
void** ybuf(eofa_net* N, int k) { return k == N->L ? &N->act[2 * N->L] : &N->yact[2 * k]; }

// output parity `parity` of layer l (adj: of its adjoint) applied to in[0..1]
void run_layer(eofa_ctx* C, eofa_net* N, int l, bool adj, void* const* in, void* out, int parity, hipStream_t st) {
  NetLayerArgs a;
  a.xin[0] = (const float*)in[0];
  a.xin[1] = (const float*)in[1];
  a.yout = (float*)out;
  a.w = N->wb + 2 * N->woff[l];
  a.links = (const float*)C->links[P32][parity];
  a.nbr = C->nbr[parity];
  a.Vh = C->g.Vh;
  a.Ls = C->g.Ls;
  a.Cin = adj ? N->ch[l + 1] : N->ch[l];
  a.Cout = adj ? N->ch[l] : N->ch[l + 1];
  a.parity = parity;
  launch_pt_layer(a, adj, st);
}

// dL/dW_l* (+)= sum_x <S_t x_ci, g_c> over both parities
void run_wgrad(eofa_ctx* C, eofa_net* N, int l, void* const* x, void* const* g, bool accumulate, hipStream_t st) {
  NetGradArgs ga;
  for (int p = 0; p < 2; ++p) {
    ga.x[p] = (const float*)x[p];
    ga.g[p] = (const float*)g[p];
    ga.links[p] = (const float*)C->links[P32][p];
    ga.nbr[p] = C->nbr[p];
  }
  ga.partial = N->partial;
  ga.Vh = C->g.Vh;
  ga.Ls = C->g.Ls;
  ga.Cin = N->ch[l];
  ga.Cout = N->ch[l + 1];
  launch_pt_wgrad(ga, WGRAD_BLOCKS, accumulate ? 1 : 0, N->gw + 2 * N->woff[l], st);
}

// N = B^dag B from act[0] (odd = input, even = 0): X[1..L] on both
// parities, then Y[L-1..0] (Y[0] on the odd parity only)
void forward(eofa_ctx* C, eofa_net* N, hipStream_t st) {
  for (int l = 0; l < N->L; ++l)
    for (int p = 0; p < 2; ++p) run_layer(C, N, l, false, &N->act[2 * l], N->act[2 * (l + 1) + p], p, st);
  for (int k = N->L; k >= 1; --k)
    for (int p = 0; p < 2; ++p) {
      if (k == 1 && p == 0) continue;
      run_layer(C, N, k - 1, true, ybuf(N, k), N->yact[2 * (k - 1) + p], p, st);
    }
}

}  // namespace

namespace eofa {

// z = N(r) for odd-sublattice packed FP32 one-channel fields
int net_apply_internal(eofa_ctx* C, eofa_net* N, const void* in, void* out, hipStream_t st) {
  NCHK(ensure_acts(C, N, st));
  const size_t hb = half_bytes(C->g, 1);
  NHIP(hipMemcpyAsync(N->act[1], in, hb, hipMemcpyDeviceToDevice, st));
  NHIP(hipMemcpyAsync(N->act[0], N->zero, hb, hipMemcpyDeviceToDevice, st));
  forward(C, N, st);
  NHIP(hipMemcpyAsync(out, N->yact[1], hb, hipMemcpyDeviceToDevice, st));
  NHIP(hipGetLastError());
  return EOFA_OK;
}

}  // namespace eofa

namespace {

// forward + backward of one pair; gradients accumulated into N->gw (written
// by the first pair of a step). sys == nullptr: error loss |y - e|^2/|e|^2,
// its unnormalised |y - e|^2 lands in loss_dst (enorm = |e|^2); else the
// residual loss 1 - |<A y, r>|^2/(|A y|^2 |r|^2) with A = M^dag M of sys
// lands in loss_dst (enorm = |r|^2, e unused).
// Backward, with G = dL/d(output)* (odd, even zero) on channel 1:
//   B^dag layers k = 1..L:  dW_{k-1}* += <S_t G, Y[k]>,  G <- L_{k-1} G;
//   B layers k = L..1:      dW_{k-1}* += <S_t X[k-1], G>, G <- L_{k-1}^dag G.
int pair_grad(eofa_ctx* C, eofa_net* N, const eofa_system* sys, const void* r, const void* e,
              const double* enorm, bool first, double* loss_dst, hipStream_t st) {
  const Geometry& g = C->g;
  const size_t hb = half_bytes(g, 1);
  NHIP(hipMemcpyAsync(N->act[1], r, hb, hipMemcpyDeviceToDevice, st));
  NHIP(hipMemcpyAsync(N->act[0], N->zero, hb, hipMemcpyDeviceToDevice, st));
  forward(C, N, st);
  int cur = 0;
  NHIP(hipMemcpyAsync(N->gbuf[cur][0], N->zero, hb, hipMemcpyDeviceToDevice, st));
  const float* y = (const float*)N->yact[1];
  if (!sys) {
    // seed: G = (y - e)/|e|^2 on odd, 0 on even; loss = sum of partials
    const int nb =
        launch_net_loss(g.Vh, g.Ls, y, (const float*)e, (float*)N->gbuf[cur][1], enorm, loss_partial(N), st);
    launch_finalize(FIN_NORM, loss_partial(N), nb, 1, CgState{}, loss_dst, st);
  } else {
    // seed: G = A dL/da* with a = A y on odd, 0 on even
    NCHK(normal_op_fp32(C, sys, y, N->ay, st));
    launch_net_resid(g.Vh, g.Ls, (const float*)N->ay, (const float*)r, enorm, loss_partial(N), loss_dst, N->coef,
                     (float*)N->dg, st);
    NCHK(normal_op_fp32(C, sys, N->dg, N->gbuf[cur][1], st));
  }
  for (int k = 1; k <= N->L; ++k) {
    run_wgrad(C, N, k - 1, N->gbuf[cur], ybuf(N, k), !first, st);
    for (int p = 0; p < 2; ++p) run_layer(C, N, k - 1, false, N->gbuf[cur], N->gbuf[1 - cur][p], p, st);
    cur = 1 - cur;
  }
  for (int k = N->L; k >= 1; --k) {
    run_wgrad(C, N, k - 1, &N->act[2 * (k - 1)], N->gbuf[cur], true, st);
    if (k > 1) {
      for (int p = 0; p < 2; ++p) run_layer(C, N, k - 1, true, N->gbuf[cur], N->gbuf[1 - cur][p], p, st);
      cur = 1 - cur;
    }
  }
  NHIP(hipGetLastError());
  return EOFA_OK;
}

int pair_norms(eofa_ctx* C, eofa_net* N, const void* e, int npairs, hipStream_t st) {
  if (N->dev_scalars_n < (size_t)2 * npairs + 2) {
    if (N->dev_scalars) (void)hipFree(N->dev_scalars);
    N->dev_scalars_n = 2 * (size_t)npairs + 2;
    NCHK(dmalloc((void**)&N->dev_scalars, N->dev_scalars_n * sizeof(double)));
  }
  const size_t hb = half_bytes(C->g, 1);
  for (int k = 0; k < npairs; ++k) {
    const int nb = launch_norm2(P32, C->g, (const char*)e + k * hb, 1, N->partial, st);
    launch_finalize(FIN_NORM, N->partial, nb, 1, CgState{}, N->dev_scalars + k, st);
  }
  NHIP(hipGetLastError());
  return EOFA_OK;
}

bool valid_channels(int L, const int32_t* ch) {
  if (L < 1 || L > 16 || !ch) return false;
  if (ch[0] != 1 || ch[L] != 1) return false;
  for (int l = 0; l <= L; ++l)
    if (ch[l] < 1 || ch[l] > NET_MAXC) return false;
  return true;
}

}  // namespace

extern "C" {

int eofa_net_create(eofa_ctx* C, int32_t n_layers, const int32_t* channels, uint64_t seed, double init_scale,
                    eofa_net** out) {
  if (!C || !out) return nfail(EOFA_ERR_INVALID, "eofa_net_create: NULL argument");
  if (!valid_channels(n_layers, channels))
    return nfail(EOFA_ERR_INVALID, "channels must run 1 -> ... -> 1 with 1..8 channels per layer");
  eofa_net* N = new eofa_net();
  N->L = n_layers;
  N->ch.assign(channels, channels + n_layers + 1);
  for (int l = 0; l < n_layers; ++l) {
    N->woff.push_back(N->nw);
    N->nw += (size_t)NET_TERMS * channels[l] * channels[l + 1];
  }
  // host initialisation: N(0, s^2) real and imaginary parts with
  // s = init_scale / sqrt(20 C_in) (splitmix64 + Box-Muller, seeded), plus
  // the identity P_+ + P_- from channel 0 to channel 0 of every layer
  std::vector<float> w(2 * N->nw);
  uint64_t state = seed;
  auto next = [&]() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  for (int l = 0; l < n_layers; ++l) {
    const double sd = init_scale / std::sqrt((double)NET_TERMS * channels[l]);
    for (size_t k = 0; k < (size_t)NET_TERMS * channels[l] * channels[l + 1]; ++k) {
      const double u1 = unif(), u2 = unif();
      const double rad = std::sqrt(-2.0 * std::log(u1));
      w[2 * (N->woff[l] + k)] = (float)(sd * rad * std::cos(2 * M_PI * u2));
      w[2 * (N->woff[l] + k) + 1] = (float)(sd * rad * std::sin(2 * M_PI * u2));
    }
    // W[t][0][0] of t = 0 (P_+) and t = 1 (P_-)
    w[2 * N->woff[l]] += 1.0f;
    w[2 * (N->woff[l] + (size_t)channels[l] * channels[l + 1])] += 1.0f;
  }
  const size_t nf = 2 * N->nw;
  if (dmalloc((void**)&N->w32, nf * 4) || dmalloc((void**)&N->m, nf * 4) || dmalloc((void**)&N->v, nf * 4) ||
      dmalloc((void**)&N->wb, nf * 2) || dmalloc((void**)&N->gw, nf * 8)) {
    eofa_net_destroy(N);
    return EOFA_ERR_OOM;
  }
  if (hipMemcpy(N->w32, w.data(), nf * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(N->m, 0, nf * 4) != hipSuccess || hipMemset(N->v, 0, nf * 4) != hipSuccess) {
    eofa_net_destroy(N);
    return nfail(EOFA_ERR_HIP, "network initialisation copy failed");
  }
  launch_net_to_bf16((int)nf, N->w32, N->wb, nullptr);
  if (hipDeviceSynchronize() != hipSuccess) {
    eofa_net_destroy(N);
    return nfail(EOFA_ERR_HIP, "network initialisation failed");
  }
  *out = N;
  return EOFA_OK;
}

int eofa_net_destroy(eofa_net* N) {
  if (!N) return EOFA_OK;
  free_acts(N);
  for (void* p : {(void*)N->w32, (void*)N->m, (void*)N->v, (void*)N->wb, (void*)N->gw, (void*)N->partial,
                  (void*)N->dev_scalars})
    if (p) (void)hipFree(p);
  delete N;
  return EOFA_OK;
}

size_t eofa_net_num_weights(const eofa_net* N) { return N ? N->nw : 0; }

int eofa_net_get_weights(const eofa_net* N, double* out) {
  if (!N || !out) return nfail(EOFA_ERR_INVALID, "eofa_net_get_weights: NULL argument");
  std::vector<float> w(2 * N->nw);
  NHIP(hipMemcpy(w.data(), N->w32, w.size() * 4, hipMemcpyDeviceToHost));
  for (size_t k = 0; k < w.size(); ++k) out[k] = w[k];
  return EOFA_OK;
}

int eofa_net_set_weights(eofa_net* N, const double* in) {
  if (!N || !in) return nfail(EOFA_ERR_INVALID, "eofa_net_set_weights: NULL argument");
  std::vector<float> w(2 * N->nw);
  for (size_t k = 0; k < w.size(); ++k) w[k] = (float)in[k];
  NHIP(hipMemcpy(N->w32, w.data(), w.size() * 4, hipMemcpyHostToDevice));
  NHIP(hipMemset(N->m, 0, w.size() * 4));
  NHIP(hipMemset(N->v, 0, w.size() * 4));
  N->step = 0;
  launch_net_to_bf16((int)w.size(), N->w32, N->wb, nullptr);
  NHIP(hipDeviceSynchronize());
  return EOFA_OK;
}

int eofa_net_apply(eofa_ctx* C, eofa_net* N, const void* in, void* out, void* stream) {
  if (!C || !N || !in || !out) return nfail(EOFA_ERR_INVALID, "eofa_net_apply: NULL argument");
  if (in == out) return nfail(EOFA_ERR_INVALID, "eofa_net_apply: in and out alias");
  return net_apply_internal(C, N, in, out, (hipStream_t)stream);
}

int eofa_net_loss_grad(eofa_ctx* C, eofa_net* N, const eofa_system* sys, const void* r, const void* e,
                       int32_t npairs, double* loss, double* grad, void* stream) {
  if (!C || !N || !r || (!e && !sys) || npairs < 1)
    return nfail(EOFA_ERR_INVALID, "eofa_net_loss_grad: bad argument");
  hipStream_t st = (hipStream_t)stream;
  NCHK(ensure_acts(C, N, st));
  NCHK(pair_norms(C, N, sys ? r : e, npairs, st));
  const size_t hb = half_bytes(C->g, 1);
  double* losses;
  NCHK(dmalloc((void**)&losses, sizeof(double) * npairs));
  for (int k = 0; k < npairs; ++k) {
    const int rc = pair_grad(C, N, sys, (const char*)r + k * hb, sys ? nullptr : (const char*)e + k * hb,
                             N->dev_scalars + k, k == 0, losses + k, st);
    if (rc != EOFA_OK) {
      (void)hipFree(losses);
      return rc;
    }
  }
  std::vector<double> lh(npairs), en(npairs);
  hipError_t e1 = hipMemcpyAsync(lh.data(), losses, sizeof(double) * npairs, hipMemcpyDeviceToHost, st);
  hipError_t e2 = hipMemcpyAsync(en.data(), N->dev_scalars, sizeof(double) * npairs, hipMemcpyDeviceToHost, st);
  hipError_t e3 = hipStreamSynchronize(st);
  (void)hipFree(losses);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return nfail(EOFA_ERR_HIP, "loss read-back failed");
  double L = 0.0;
  for (int k = 0; k < npairs; ++k) L += sys ? lh[k] : lh[k] / en[k];
  if (loss) *loss = L;
  if (grad) NHIP(hipMemcpy(grad, N->gw, sizeof(double) * 2 * N->nw, hipMemcpyDeviceToHost));
  return EOFA_OK;
}

int eofa_net_train(eofa_ctx* C, eofa_net* N, const eofa_system* sys, const void* r, const void* e, int32_t npairs,
                   int32_t epochs, int32_t batch, double lr, double* loss_per_epoch, void* stream) {
  if (!C || !N || !r || (!e && !sys) || npairs < 1 || epochs < 1 || batch < 1 || !(lr > 0.0))
    return nfail(EOFA_ERR_INVALID, "eofa_net_train: bad argument");
  hipStream_t st = (hipStream_t)stream;
  NCHK(ensure_acts(C, N, st));
  NCHK(pair_norms(C, N, sys ? r : e, npairs, st));
  const size_t hb = half_bytes(C->g, 1);
  double* losses;
  NCHK(dmalloc((void**)&losses, sizeof(double) * npairs));
  std::vector<double> lh(npairs), en(npairs);
  for (int ep = 0; ep < epochs; ++ep) {
    for (int b0 = 0; b0 < npairs; b0 += batch) {
      const int b1 = std::min(npairs, b0 + batch);
      for (int k = b0; k < b1; ++k) {
        const int rc = pair_grad(C, N, sys, (const char*)r + k * hb, sys ? nullptr : (const char*)e + k * hb,
                                 N->dev_scalars + k, k == b0, losses + k, st);
        if (rc != EOFA_OK) {
          (void)hipFree(losses);
          return rc;
        }
      }
      N->step += 1;
      launch_net_adam((int)(2 * N->nw), N->w32, N->m, N->v, N->gw, 1.0 / (b1 - b0), (float)lr, 0.9f, 0.999f,
                      1e-8f, N->step, N->wb, st);
    }
    if (hipMemcpyAsync(lh.data(), losses, sizeof(double) * npairs, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(en.data(), N->dev_scalars, sizeof(double) * npairs, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      (void)hipFree(losses);
      return nfail(EOFA_ERR_HIP, "training loss read-back failed");
    }
    double L = 0.0;
    for (int k = 0; k < npairs; ++k) L += sys ? lh[k] : lh[k] / en[k];
    if (loss_per_epoch) loss_per_epoch[ep] = L / npairs;
  }
  (void)hipFree(losses);
  NHIP(hipGetLastError());
  return EOFA_OK;
}

}  // extern "C"
