// C ABI, context and the batched CG driver (host side).
//
// Solve route (App. B, App. B.2, Sec. VI A), per right-hand side r:
//   b = g5 R5 phi                                  (eqn non_hermit_sys)
//   b~_o = b_o - M_oe M_ee^-1 b_e                  (Schur source)
//   FP64 outer loop (defect correction):
//     r_o = b~_o - M^ x_o,  stop if |r_o| <= tol |b|
//     inner CGNR on M^dag M e = M^dag r_o in the inner precision
//     x_o += e
//   psi'_e = M_ee^-1 (b_e - M_eo x_o),  psi = D~ psi'   (eqn precond_mobius_eofa_system)
// with M^ = M_ee - M_oe M_ee^-1 M_eo, M_eo = Dhop_eo D~. The odd Schur
// residual equals the full residual of the Cayley system once psi'_e is
// reconstructed, and |b| = |phi| since g5 R5 is unitary, so the outer test is
// the FP64 true residual of the EOFA system; it is re-measured on the full
// lattice at the end.
//
// Inner CGNR iteration (all right-hand sides in the same kernels, each with
// its own scalars; a right-hand side that has converged is skipped by every
// kernel through its halt flag):
//   K1  t_e = M_ee^-1 Dhop D~ p_o
//   K2  w_o = M_ee p_o - Dhop D~ t_e          |w|^2 -> alpha = |r|^2/|w|^2
//   K3  t_e = M_ee^-T D~^T Dhop^dag w_o
//   K4  r_o -= alpha (M_ee^T w_o - D~^T Dhop^dag t_e)   |r|^2 -> beta
//   U   x_o += alpha p_o,  p_o = r_o + beta p_o
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "nn_internal.h"
#include "force_internal.h"

using namespace eofa;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(EOFA_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

#define CHK(call)                \
  do {                           \
    int c_ = (call);             \
    if (c_ != EOFA_OK) return c_; \
  } while (0)

}  // namespace

int eofa::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

constexpr size_t kStageInit = size_t(1) << 20;  // pinned host staging per context

// ---------------------------------------------------------------------------
// Workspace of the no-allocation solve (eofa_cg_solve_noalloc): a file-scope
// device array of kNoallocBytes, one copy on every GPU the library runs on,
// held until the process ends. Host code never passes the array's name to a
// kernel: its device address on each GPU comes from hipGetSymbolAddress, taken
// once per device (at context creation, with that device current).
constexpr size_t kNoallocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EOFA_ERR_INVALID, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return EOFA_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(EOFA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = p;
  return EOFA_OK;
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

int ws(eofa_ctx* C, const char* name, size_t bytes, void** out) {
  if (C->arena) {  // no-allocation call: carve from the scratch array
    Arena& A = *C->arena;
    auto it = A.slots.find(name);
    if (it != A.slots.end() && it->second.second >= bytes) {
      *out = A.base + it->second.first;
      return EOFA_OK;
    }
    const size_t off = (A.used + 255) & ~size_t(255);
    if (off + bytes > A.cap)
      return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: workspace beyond its " + std::to_string(A.cap >> 20) +
                                        " MiB scratch (buffer " + name + ")");
    A.slots[name] = {off, bytes};
    A.used = off + bytes;
    *out = A.base + off;
    return EOFA_OK;
  }
  Buf& b = C->pool[name];
  if (b.n < bytes) {
    if (b.p) HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(EOFA_ERR_OOM, std::string("hipMalloc failed for workspace ") + name);
    }
    b.n = bytes;
  }
  *out = b.p;
  return EOFA_OK;
}

int stage(eofa_ctx* C, size_t bytes) {
  if (C->arena && C->host_stage_n < bytes)
    return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: host staging beyond the " +
                                      std::to_string(C->host_stage_n) + " bytes set aside at context creation");
  if (C->host_stage_n < bytes) {
    if (C->host_stage) HIPCHK(hipHostFree(C->host_stage));
    C->host_stage = nullptr;
    C->host_stage_n = 0;
    HIPCHK(hipHostMalloc((void**)&C->host_stage, bytes, hipHostMallocDefault));
    C->host_stage_n = bytes;
  }
  return EOFA_OK;
}

size_t mats_per_rhs(const Geometry& g) { return (size_t)NMAT * 2 * g.Ls * g.Ls; }
size_t scoef_per_rhs(const Geometry& g) { return (size_t)SCOEF_HEAD + 2 * (size_t)g.Ls; }

// Build and upload the fifth-dimension matrices and operator masses of
// sys[0..nrhs). Cached: a repeat of the same systems uploads nothing.
int upload_systems(eofa_ctx* C, const eofa_system* sys, int nrhs, hipStream_t st) {
  std::vector<double> key;
  key.reserve(nrhs * 5);
  for (int r = 0; r < nrhs; ++r) {
    key.push_back(sys[r].m_op);
    key.push_back(sys[r].m_a);
    key.push_back(sys[r].m_b);
    key.push_back(sys[r].beta);
    key.push_back(sys[r].beta != 0.0 ? (double)sys[r].chi : 0.0);
  }
  if (!C->arena && key == C->sys_key && C->mats) return EOFA_OK;
  const size_t per = mats_per_rhs(C->g), sper = scoef_per_rhs(C->g);
  const size_t n = per * nrhs + nrhs + sper * nrhs;
  std::vector<double> h(n);
  for (int r = 0; r < nrhs; ++r) {
    std::string err;
    const int rc = build_fifth(C->g, C->M5, C->b5, C->c5, sys[r], h.data() + per * r, err);
    if (rc != EOFA_OK) return fail(rc, "right-hand side " + std::to_string(r) + ": " + err);
    h[per * nrhs + r] = sys[r].m_op;
    build_struct(C->g, C->M5, C->b5, C->c5, sys[r], h.data() + per * nrhs + nrhs + sper * r);
  }
  if (C->arena) {  // no-allocation call: the coefficients live in the scratch array
    void* m;
    CHK(ws(C, "mats", n * sizeof(double), &m));
    CHK(stage(C, n * sizeof(double)));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(C->host_stage, h.data(), n * sizeof(double));
    HIPCHK(hipMemcpyAsync(m, C->host_stage, n * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    C->mats_active = (double*)m;
    return EOFA_OK;
  }
  if (C->mats_n < n) {
    if (C->mats) HIPCHK(hipFree(C->mats));
    C->mats = nullptr;
    if (hipMalloc((void**)&C->mats, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      C->mats_n = 0;
      return fail(EOFA_ERR_OOM, "hipMalloc failed for coefficient buffer");
    }
    C->mats_n = n;
  }
  CHK(stage(C, n * sizeof(double)));
  HIPCHK(hipStreamSynchronize(st));  // the staging buffer may still feed an earlier copy
  std::memcpy(C->host_stage, h.data(), n * sizeof(double));
  HIPCHK(hipMemcpyAsync(C->mats, C->host_stage, n * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  C->sys_key = key;
  return EOFA_OK;
}

// the coefficients of the systems last uploaded (the scratch copy during a
// no-allocation call)
double* mats_of(eofa_ctx* C) { return C->mats_active ? C->mats_active : C->mats; }
const double* mop_ptr(eofa_ctx* C, int nrhs) { return mats_of(C) + mats_per_rhs(C->g) * nrhs; }

int check_prec(int prec) {
  if (prec < 0 || prec > 2) return fail(EOFA_ERR_INVALID, "precision must be EOFA_FP64, EOFA_FP32 or EOFA_FP16S");
  return EOFA_OK;
}

int check_systems(const eofa_system* sys, int nrhs) {
  if (!sys) return fail(EOFA_ERR_INVALID, "sys is NULL");
  if (nrhs < 1) return fail(EOFA_ERR_INVALID, "nrhs must be >= 1");
  for (int r = 0; r < nrhs; ++r) {
    if (sys[r].beta != 0.0 && sys[r].chi != 1 && sys[r].chi != -1)
      return fail(EOFA_ERR_INVALID, "eofa_system.chi must be +1 or -1");
    if (!std::isfinite(sys[r].m_op) || !std::isfinite(sys[r].beta) || !std::isfinite(sys[r].m_a) ||
        !std::isfinite(sys[r].m_b))
      return fail(EOFA_ERR_INVALID, "non-finite system parameter");
  }
  return EOFA_OK;
}

HopArgs base_args(eofa_ctx* C, int prec, int out_parity, int nrhs) {
  HopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.links = C->links[prec][out_parity];
  a.nbr = C->nbr[out_parity];
  a.order = C->order;
  a.mats = mats_of(C);
  a.matA = 0;
  a.matB = 0;
  a.cpd = C->c + C->d;
  a.cmd = C->c - C->d;
  a.mop = mop_ptr(C, nrhs);
  a.scoef = mop_ptr(C, nrhs) + nrhs;
  a.bee = (C->c + C->d) * (4.0 - C->M5) + 1.0;
  a.cee = 1.0 - (C->c - C->d) * (4.0 - C->M5);
  a.Vh = C->g.Vh;
  a.Ls = C->g.Ls;
  a.nrhs = nrhs;
  a.rhs_block = nrhs;
  a.W = default_waves(C->g.Ls);
  auto it = C->tuned.find(prec * 4096 + nrhs);
  if (it != C->tuned.end()) {
    a.W = it->second.first;
    a.rhs_block = it->second.second;
  }
  return a;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char* eofa_last_error(void) { return g_err.c_str(); }

int eofa_create(const eofa_action* act, const void* gauge, void* stream, eofa_ctx** out) {
  if (!act || !gauge || !out) return fail(EOFA_ERR_INVALID, "eofa_create: NULL argument");
  *out = nullptr;
  for (int k = 0; k < 4; ++k) {
    if (act->dims[k] < 2 || act->dims[k] % 2 != 0)
      return fail(EOFA_ERR_INVALID, "every lattice extent must be even and >= 2");
    const bool gp_ok = k == 0 && act->bc[k] == 2;
    if (act->bc[k] != 1 && act->bc[k] != -1 && !gp_ok)
      return fail(EOFA_ERR_INVALID, "bc entries must be +1 or -1 (bc[0] may be 2: G-parity in x)");
  }
  const bool gparity = act->bc[0] == 2;
  if (act->Ls < 2 || act->Ls > 32 || act->Ls % 2 != 0) return fail(EOFA_ERR_INVALID, "Ls must be even, 2..32");
  if (std::fabs(act->b5 - act->c5 - 1.0) > 1e-12)
    return fail(EOFA_ERR_INVALID, "b5 - c5 must be 1 (d = 1/2)");
  if (!std::isfinite(act->M5) || !std::isfinite(act->b5) || !std::isfinite(act->c5))
    return fail(EOFA_ERR_INVALID, "non-finite action parameter");
  const double V = (double)act->dims[0] * act->dims[1] * act->dims[2] * act->dims[3] * (gparity ? 2 : 1);
  // 32-bit site indexing, and the FP16S gathers' 32-bit byte offsets within
  // one quad plane (16 bytes per 5D site of a parity)
  if (V / 2 * act->Ls * 6 > 2.0e9 || V / 2 * act->Ls * 16 >= 4294967296.0)
    return fail(EOFA_ERR_INVALID, "lattice too large for 32-bit indexing (Vh * Ls must stay below 2^28)");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(EOFA_ERR_INVALID, std::string("this library is built for gfx950; device is ") + prop.gcnArchName);

  CHK(scratch_init(dev));
  eofa_ctx* C = new eofa_ctx();
  C->device = dev;
  // host staging set aside now, so that the no-allocation solve needs none
  if (hipHostMalloc((void**)&C->host_stage, kStageInit, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    C->host_stage = nullptr;
    eofa_destroy(C);
    return fail(EOFA_ERR_OOM, "hipHostMalloc failed for the host staging buffer");
  }
  C->host_stage_n = kStageInit;
  for (int k = 0; k < 4; ++k) {
    C->g.L[k] = act->dims[k];
    C->bc[k] = act->bc[k];
  }
  if (gparity) {  // x-doubled lattice, flavour-1 copy at x + Lx, antiperiodic x edge
    C->gparity = true;
    C->Lx_phys = act->dims[0];
    C->g.L[0] = 2 * act->dims[0];
    C->bc[0] = -1;
  }
  C->g.Ls = act->Ls;
  C->g.V = (int)V;
  C->g.Vh = (int)(V / 2);
  C->M5 = act->M5;
  C->b5 = act->b5;
  C->c5 = act->c5;
  C->c = 0.5 * (act->b5 + act->c5);
  C->d = 0.5 * (act->b5 - act->c5);
  hipStream_t st = (hipStream_t)stream;
  for (int p = 0; p < 3; ++p)
    for (int par = 0; par < 2; ++par)
      if (hipMalloc(&C->links[p][par], link_bytes(p, C->g)) != hipSuccess) {
        (void)hipGetLastError();
        eofa_destroy(C);
        return fail(EOFA_ERR_OOM, "hipMalloc failed for links");
      }
  for (int par = 0; par < 2; ++par)
    if (hipMalloc((void**)&C->nbr[par], (size_t)C->g.Vh * 8 * sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      eofa_destroy(C);
      return fail(EOFA_ERR_OOM, "hipMalloc failed for neighbour table");
    }
  if (hipMalloc((void**)&C->order, (size_t)C->g.Vh * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    eofa_destroy(C);
    return fail(EOFA_ERR_OOM, "hipMalloc failed for the traversal order");
  }
  {
    std::vector<int> ord(C->g.Vh);
    site_order(C->g, ord.data());
    if (hipMemcpy(C->order, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      eofa_destroy(C);
      return fail(EOFA_ERR_HIP, "traversal order upload failed");
    }
  }
  void* l64[2] = {C->links[P64][0], C->links[P64][1]};
  void* l32[2] = {C->links[P32][0], C->links[P32][1]};
  void* l16[2] = {C->links[P16][0], C->links[P16][1]};
  void* gauge2 = nullptr;
  if (gparity) {
    const size_t rows = (size_t)C->g.L[1] * C->g.L[2] * C->g.L[3];
    if (hipMalloc(&gauge2, (size_t)4 * rows * C->g.L[0] * 9 * 16) != hipSuccess) {
      (void)hipGetLastError();
      eofa_destroy(C);
      return fail(EOFA_ERR_OOM, "hipMalloc failed for the x-doubled gauge field");
    }
    launch_double_gauge(C->Lx_phys, rows, gauge, gauge2, st);
  }
  launch_gauge_pack(C->g, gparity ? gauge2 : gauge, C->bc, l64, l32, l16, C->nbr, st);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipGetLastError();
  if (gauge2) (void)hipFree(gauge2);
  if (e != hipSuccess) {
    eofa_destroy(C);
    return fail(EOFA_ERR_HIP, std::string("gauge packing: ") + hipGetErrorString(e));
  }
  *out = C;
  return EOFA_OK;
}

int eofa_destroy(eofa_ctx* C) {
  if (!C) return EOFA_OK;
  for (int p = 0; p < 3; ++p)
    for (int par = 0; par < 2; ++par)
      if (C->links[p][par]) (void)hipFree(C->links[p][par]);
  for (int par = 0; par < 2; ++par)
    if (C->nbr[par]) (void)hipFree(C->nbr[par]);
  if (C->order) (void)hipFree(C->order);
  for (auto& kv : C->pool)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (C->mats) (void)hipFree(C->mats);
  if (C->host_stage) (void)hipHostFree(C->host_stage);
  for (auto ev : C->events) (void)hipEventDestroy(ev);
  if (C->cap_stream) (void)hipStreamDestroy(C->cap_stream);
  delete C;
  return EOFA_OK;
}

size_t eofa_packed_bytes(const eofa_ctx* C, int32_t prec, int32_t nrhs) {
  if (!C || prec < 0 || prec > 2 || nrhs < 1) return 0;
  return packed_bytes(prec, C->g, nrhs);
}

int eofa_pack(eofa_ctx* C, const void* full, void* packed, int32_t parity, int32_t prec, int32_t nrhs,
              int32_t g5r5, void* stream) {
  if (!C || !full || !packed) return fail(EOFA_ERR_INVALID, "eofa_pack: NULL argument");
  if (parity != 0 && parity != 1) return fail(EOFA_ERR_INVALID, "parity must be 0 or 1");
  if (nrhs < 1) return fail(EOFA_ERR_INVALID, "nrhs must be >= 1");
  CHK(check_prec(prec));
  launch_pack(prec, C->g, full, packed, parity, nrhs, g5r5 ? 1 : 0, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

int eofa_unpack(eofa_ctx* C, const void* packed, void* full, int32_t parity, int32_t prec, int32_t nrhs,
                void* stream) {
  if (!C || !full || !packed) return fail(EOFA_ERR_INVALID, "eofa_unpack: NULL argument");
  if (parity != 0 && parity != 1) return fail(EOFA_ERR_INVALID, "parity must be 0 or 1");
  if (nrhs < 1) return fail(EOFA_ERR_INVALID, "nrhs must be >= 1");
  CHK(check_prec(prec));
  launch_unpack(prec, C->g, packed, full, parity, nrhs, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

int eofa_dslash(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, int32_t out_parity,
                int32_t dagger, int32_t prec, int32_t nrhs, void* stream) {
  if (!C || !in || !out) return fail(EOFA_ERR_INVALID, "eofa_dslash: NULL argument");
  if (in == out) return fail(EOFA_ERR_INVALID, "eofa_dslash: in and out alias");
  if (out_parity != 0 && out_parity != 1) return fail(EOFA_ERR_INVALID, "parity must be 0 or 1");
  CHK(check_prec(prec));
  CHK(check_systems(sys, nrhs));
  hipStream_t st = (hipStream_t)stream;
  CHK(upload_systems(C, sys, nrhs, st));
  HopArgs a = base_args(C, prec, out_parity, nrhs);
  a.in = in;
  a.out = out;
  a.matA = MAT_DT_T;
  const int rc = launch_hop(prec, dagger ? ROLE_DSLASH_DAG : ROLE_DSLASH, a, st, nullptr);
  if (rc != EOFA_OK) return fail(rc, std::string("hop kernel launch: ") + hipGetErrorString(hipGetLastError()));
  return EOFA_OK;
}

static int smat_entry(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, int mat, int prec,
                      int nrhs, void* stream) {
  if (!C || !in || !out) return fail(EOFA_ERR_INVALID, "NULL argument");
  if (in == out) return fail(EOFA_ERR_INVALID, "in and out alias");
  CHK(check_prec(prec));
  CHK(check_systems(sys, nrhs));
  hipStream_t st = (hipStream_t)stream;
  CHK(upload_systems(C, sys, nrhs, st));
  launch_smat(prec, C->g, in, out, mats_of(C), mat, nrhs, st);
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

int eofa_mooee(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, int32_t dagger, int32_t prec,
               int32_t nrhs, void* stream) {
  return smat_entry(C, sys, in, out, dagger ? MAT_MEE_T : MAT_MEE, prec, nrhs, stream);
}

int eofa_mooee_inv(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, int32_t dagger,
                   int32_t prec, int32_t nrhs, void* stream) {
  return smat_entry(C, sys, in, out, dagger ? MAT_MEE_INV_T : MAT_MEE_INV, prec, nrhs, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solve

namespace {

struct Scal {
  CgState s;
  void* base = nullptr;
};

int alloc_state(eofa_ctx* C, int nrhs, CgState& S) {
  void* b = nullptr;
  const size_t nd = 8, ni = 5;
  CHK(ws(C, "cgstate", (nd * sizeof(double) + ni * sizeof(int)) * nrhs + 64, &b));
  double* d = (double*)b;
  S.rr = d;
  S.stop = d + nrhs;
  S.ww = d + 2 * nrhs;
  S.alpha = d + 3 * nrhs;
  S.beta = d + 4 * nrhs;
  S.tol2 = d + 5 * nrhs;
  S.norm = d + 6 * nrhs;
  S.guard = d + 7 * nrhs;
  int* ip = (int*)(d + nd * nrhs);
  S.iter = ip;
  S.max_iter = ip + nrhs;
  S.halt = ip + 2 * nrhs;
  S.u2run = ip + 3 * nrhs;
  S.breakdown = ip + 4 * nrhs;
  return EOFA_OK;
}

int hop(eofa_ctx* C, int prec, int role, HopArgs a, hipStream_t st, int* nblk = nullptr) {
  const int rc = launch_hop(prec, role, a, st, nblk);
  if (rc != EOFA_OK) return fail(rc, std::string("hop kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
  return EOFA_OK;
}

// device norms |f|^2 per rhs -> host out[nrhs] (synchronises)
int norms(eofa_ctx* C, int prec, const void* f, int nrhs, double* partial, CgState S, std::vector<double>& out,
          hipStream_t st) {
  const int nb = launch_norm2(prec, C->g, f, nrhs, partial, st);
  launch_finalize(FIN_NORM, partial, nb, nrhs, S, S.norm, st);
  out.resize(nrhs);
  HIPCHK(hipMemcpyAsync(C->host_stage, S.norm, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(out.data(), C->host_stage, nrhs * sizeof(double));
  return EOFA_OK;
}

int fetch(eofa_ctx* C, const void* dev, size_t bytes, void* host, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(C->host_stage, dev, bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(host, C->host_stage, bytes);
  return EOFA_OK;
}

int put(eofa_ctx* C, void* dev, const void* host, size_t bytes, hipStream_t st) {
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(C->host_stage, host, bytes);
  HIPCHK(hipMemcpyAsync(dev, C->host_stage, bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return EOFA_OK;
}

// The kernels and fifth-dimension matrices of one form of the odd Schur
// system. Cayley (App. B.2): off-parity blocks Dhop D~, same-parity M_ee.
// Dense (the EOFA matrix itself, for comparison): off-parity blocks Dhop,
// same-parity D_ee = M_ee D~^-1, both forms with the same residual b - D psi.
// Cayley form: the inner CG holds its search direction as p~ = D~ p, so K1
// gathers an already premixed field (no D~ on its 8 neighbour columns), K2
// applies M_ee D~^-1 to the same-site p~, the update forms D~ r by lane
// exchange, and the solution accumulates x~ = D~ x (D~^-1 once per pass).
struct Form {
  int k1, k2, k3, k4, k4s, src, res, fullres;  // roles (k1, k2 of the inner iteration)
  int m1, m2, m3, m4a, m4b;                     // matA of K1, matB of K2, matA of K3, matA/matB of K4
  int inv, diag;                                // same-parity block inverse / block (source, residual)
  bool cayley;                                  // psi = D~ psi' on reconstruction, guess through D~^-1
  int k1x;                                      // K1 on a plain (not premixed) x: the FP64 outer residual
  bool ptilde;                                  // inner direction held as p~ = D~ p
};
const Form kCayley = {ROLE_K1T, ROLE_K2T, ROLE_K3, ROLE_K4, ROLE_K4S, ROLE_SRC, ROLE_RES, ROLE_FULLRES,
                      MAT_MEE_INV, MAT_MEE, MAT_MEE_INV_T, MAT_NEG_DT_T, MAT_MEE_T,
                      MAT_MEE_INV, MAT_MEE, true, ROLE_K1, true};
const Form kDense = {ROLE_D1, ROLE_D2, ROLE_D3, ROLE_D4, ROLE_D4S, ROLE_DSRC, ROLE_DRES, ROLE_DFULLRES,
                     MAT_DEE_INV, MAT_DEE, MAT_DEE_INV_T, 0, MAT_DEE_T,
                     MAT_DEE_INV, MAT_DEE, false, ROLE_D1, false};

DtArgs dt_args(eofa_ctx* C, const Form& F, int nrhs) {
  DtArgs d;
  if (F.ptilde) {
    d.mop = mop_ptr(C, nrhs);
    d.cpd = C->c + C->d;
    d.cmd = C->c - C->d;
  }
  return d;
}

// Ring of search directions for the batched solution update: iteration k
// reads p_k from slot k mod R and writes p_{k+1} to the next slot; every
// F = R / 2 iterations x += sum alpha_j p_j over the last F slots (one pass
// over x per F iterations instead of one per iteration). R (16, 8 or 4)
// divides the host poll and graph period, so slot indices repeat
// identically in every replay.
struct Ring {
  char* base = nullptr;
  size_t slot = 0;           // bytes per slot (all right-hand sides)
  double* ahist = nullptr;   // [R][nrhs] alpha of each step, 0 if it did not run
  int R = 16, F = 8;
  void* at(int k) const { return base + (size_t)(k % R) * slot; }
};

// One inner CGNR iteration k: K1, K2, alpha, K3, K4, beta, x/p update, all on
// one stream (the alpha finalize on a second stream beside K3 cost two
// cross-stream waits, about 6 us each, more than the finalize itself).
int inner_iteration(eofa_ctx* C, const Form& F, int S, const HopArgs& k1, const HopArgs& k2,
                    const HopArgs& k3, const HopArgs& k4, int nbh, int nrhs, CgState Sst, double* partial,
                    void* xin, void* rin, void* pS, hipStream_t st, hipEvent_t* ev, const Ring* ring, int k) {
  const Geometry& g = C->g;
  HopArgs a1 = k1, a2 = k2;
  if (ring) a1.in = a2.y = ring->at(k);
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  CHK(hop(C, S, F.k1, a1, st));
  if (ev) HIPCHK(hipEventRecord(ev[1], st));
  if (ev) HIPCHK(hipEventRecord(ev[2], st));
  CHK(hop(C, S, F.k2, a2, st));
  if (ev) HIPCHK(hipEventRecord(ev[3], st));
  // the alpha step on K2's partial sums runs in K3's work-group 0 (K3 does
  // not need alpha; K4, the launch after it, does) when that work-group can
  // sum them with at most 16 loads per thread; else (small work-groups, many
  // partials) in a finalize launch of its own
  HopArgs a3 = k3;
  if (nbh <= 16 * 64 * k3.W) {
    a3.fin_partial = partial;
    a3.fin_nblk = nbh;
    a3.fin_mode = FIN_ALPHA;
    a3.fin_S = Sst;
  } else {
    launch_finalize(FIN_ALPHA, partial, nbh, nrhs, Sst, nullptr, st);
  }
  if (ev) HIPCHK(hipEventRecord(ev[4], st));
  CHK(hop(C, S, F.k3, a3, st));
  if (ev) HIPCHK(hipEventRecord(ev[5], st));
  if (ev) HIPCHK(hipEventRecord(ev[6], st));
  CHK(hop(C, S, F.k4, k4, st));
  if (ev) HIPCHK(hipEventRecord(ev[7], st));
  launch_finalize(FIN_BETA, partial, nbh, nrhs, Sst, nullptr, st);
  const DtArgs dt = dt_args(C, F, nrhs);
  if (ring) {
    launch_p_update(S, g, rin, ring->at(k), ring->at(k + 1), Sst.alpha, Sst.beta, Sst.u2run,
                    ring->ahist + (size_t)(k % ring->R) * nrhs, nrhs, dt, st);
    if ((k + 1) % ring->F == 0)
      launch_x_flush(S, g, xin, ring->base, ring->slot, (k + 1 - ring->F) % ring->R, ring->F, ring->R, ring->ahist,
                     nrhs, st);
  } else {
    launch_cg_update(S, g, xin, rin, pS, Sst.alpha, Sst.beta, Sst.u2run, nrhs, dt, st);
  }
  return EOFA_OK;
}

// Autotuner: time the four inner hop kernels for each (waves per
// work-group, right-hand sides per work-group) candidate on the solve's own
// buffers (halt flags off, before the CG state exists) and keep the fastest
// (best of three timed passes per candidate). Picks are kept per context
// and in a process-wide cache keyed by device, lattice and the context key,
// so a later context of the same shape does not tune again.
int tune_key(const Form& F, int S, int nrhs) { return ((F.cayley ? 0 : 8) + S) * 4096 + nrhs; }

std::mutex g_tune_mu;
std::map<std::vector<int>, std::pair<int, int>> g_tune_cache;

std::vector<int> tune_cache_key(const eofa_ctx* C, int key) {
  return {C->device, C->g.L[0], C->g.L[1], C->g.L[2], C->g.L[3], C->g.Ls, key};
}

int autotune(eofa_ctx* C, const Form& F, int S, int nrhs, HopArgs k1, HopArgs k2, HopArgs k3, HopArgs k4,
             hipStream_t st) {
  const int key = tune_key(F, S, nrhs);
  if (C->tuned.count(key)) return EOFA_OK;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune_cache.find(tune_cache_key(C, key));
    if (it != g_tune_cache.end()) {
      C->tuned[key] = it->second;
      return EOFA_OK;
    }
  }
  const int Ls = C->g.Ls;
  std::vector<int> waves, blocks;
  for (int w : {1, 2, 4}) {
    bool fits = true;
    for (int role : {F.k1, F.k2, F.k3, F.k4})
      fits = fits && hop_lds_bytes(S, role, Ls, w) <= 65536;
    if (fits) waves.push_back(w);
  }
  for (int rb = 1; rb <= nrhs; ++rb)
    if (rb == nrhs || (nrhs + rb - 1) / rb != (nrhs + rb) / (rb + 1)) blocks.push_back(rb);
  if (waves.empty()) waves.push_back(default_waves(Ls));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best = 1e30;
  std::pair<int, int> pick(default_waves(Ls), nrhs);
  for (int w : waves)
    for (int rb : blocks) {
      HopArgs a[4] = {k1, k2, k3, k4};
      for (auto& x : a) {
        x.W = w;
        x.rhs_block = rb;
        x.halt = nullptr;
      }
      const int roles[4] = {F.k1, F.k2, F.k3, F.k4};
      for (int k = 0; k < 4; ++k) CHK(hop(C, S, roles[k], a[k], st));  // warm-up
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(hipEventRecord(e0, st));
        for (int k = 0; k < 4; ++k) CHK(hop(C, S, roles[k], a[k], st));
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          pick = {w, rb};
        }
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  C->tuned[key] = pick;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[tune_cache_key(C, key)] = pick;
  return EOFA_OK;
}

// psi'_e = M_ee^-1 (b_e - Dhop D~ x_o), the FP64 true residual of the
// Cayley system per parity (re, rodd: |.|^2 per rhs), psi = D~ psi' unpacked
// to the canonical layout (dense form: psi_e = D_ee^-1 (b_e - Dhop x_o), psi
// itself unpacked). Overwrites te, tmp, ro; synchronises.
int reconstruct(eofa_ctx* C, const Form& F, int nrhs, void* x, void* be, void* bo, void* te, void* tmp, void* ro,
                double* partial, CgState Sst, void* psi, std::vector<double>& re, std::vector<double>& rodd,
                hipStream_t st) {
  const Geometry& g = C->g;
  re.assign(nrhs, 0.0);
  rodd.assign(nrhs, 0.0);
  // reconstruct psi'_e = M_ee^-1 (b_e - Dhop D~ x_o)
  {
    HopArgs a = base_args(C, P64, 0, nrhs);
    a.in = x;
    a.z = be;
    a.out = tmp;
    CHK(hop(C, P64, F.src, a, st));
  }
  launch_smat(P64, g, tmp, te, mats_of(C), F.inv, nrhs, st);
  // FP64 true residual of the system on both parities
  {
    HopArgs a = base_args(C, P64, 0, nrhs);
    a.in = x;
    a.y = te;
    a.z = be;
    a.out = tmp;
    a.matB = F.diag;
    a.partial = partial;
    int nb = 0;
    CHK(hop(C, P64, F.fullres, a, st, &nb));
    launch_finalize(FIN_NORM, partial, nb, nrhs, Sst, Sst.norm, st);
    CHK(fetch(C, Sst.norm, nrhs * sizeof(double), re.data(), st));
    HopArgs b = base_args(C, P64, 1, nrhs);
    b.in = te;
    b.y = x;
    b.z = bo;
    b.out = ro;
    b.matB = F.diag;
    b.partial = partial;
    CHK(hop(C, P64, F.fullres, b, st, &nb));
    launch_finalize(FIN_NORM, partial, nb, nrhs, Sst, Sst.norm, st);
    CHK(fetch(C, Sst.norm, nrhs * sizeof(double), rodd.data(), st));
  }
  if (F.cayley) {  // psi = D~ psi'
    launch_smat(P64, g, te, tmp, mats_of(C), MAT_DT, nrhs, st);
    launch_unpack(P64, g, tmp, psi, 0, nrhs, st);
    launch_smat(P64, g, x, ro, mats_of(C), MAT_DT, nrhs, st);
    launch_unpack(P64, g, ro, psi, 1, nrhs, st);
  } else {
    launch_unpack(P64, g, te, psi, 0, nrhs, st);
    launch_unpack(P64, g, x, psi, 1, nrhs, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

// tolr: per right-hand side FP64 true-residual targets (nullptr: prm->tol for all)
int solve_batch(eofa_ctx* C, const eofa_system* sys, int nrhs, const void* phi, void* psi,
                const eofa_solver_params* prm, eofa_solver_stats* stats, hipStream_t st,
                const double* tolr = nullptr) {
  const double t0 = now_s();
  const Geometry& g = C->g;
  const Form& F = prm->form == 1 ? kDense : kCayley;
  const int S = prm->inner_prec;
  // the inner residual is kept in the inner precision S, the inner
  // solution in FP32 (FP64 for FP64 inner solves)
  const int PX = S == P64 ? P64 : P32;
  const bool fixed = prm->fixed_iters > 0;
  const int max_outer = fixed ? 1 : std::max(1, prm->max_outer);
  const int check = prm->check_every > 0 ? prm->check_every : 16;
  // Each inner pass aims only at the reduction still missing (0.3 safety
  // factor on the FP64 target), floored at the inner precision's reach.
  double inner_floor = prm->inner_tol;
  if (!(inner_floor > 0.0)) inner_floor = S == P64 ? 0.0 : 1e-4;
  // A kept direction stays conjugate only while the inner recurrence
  // residual is close to the true one, i.e. when each pass reduces the
  // residual by a factor well above the inner precision's unit roundoff
  // (2^-11 FP16S, 2^-24 FP32): replace the residual every 10x (FP16S) or
  // 100x (FP32) of reduction.
  const bool keep = prm->keep_direction && S != P64 && !fixed;
  if (keep) inner_floor = std::max(inner_floor, S == P16 ? 0.1 : 0.01);

  CHK(upload_systems(C, sys, nrhs, st));
  CHK(stage(C, 64 * (size_t)std::max(nrhs, 16)));
  const size_t b64 = packed_bytes(P64, g, nrhs), bS = packed_bytes(S, g, nrhs), bX = packed_bytes(PX, g, nrhs);
  void *be, *bo, *bt, *x, *ro, *te, *tmp, *rS, *pS, *tS, *wS, *rin, *xin, *partial_v;
  CHK(ws(C, "be", b64, &be));
  CHK(ws(C, "bo", b64, &bo));
  CHK(ws(C, "bt", b64, &bt));
  CHK(ws(C, "x", b64, &x));
  CHK(ws(C, "ro", b64, &ro));
  CHK(ws(C, "te", b64, &te));
  CHK(ws(C, "tmp", b64, &tmp));
  CHK(ws(C, "rS", bS, &rS));
  CHK(ws(C, "pS", bS, &pS));
  CHK(ws(C, "tS", bS, &tS));
  CHK(ws(C, "wS", bS, &wS));
  CHK(ws(C, "rin", bS, &rin));
  CHK(ws(C, "xin", bX, &xin));
  const int maxblk = std::max(hop_blocks(P64, g.Vh, g.Ls, 1), (g.Ls * g.Vh + 255) / 256);  // W = 1 has the most blocks
  CHK(ws(C, "partial", sizeof(double) * (size_t)maxblk * nrhs, &partial_v));
  double* partial = (double*)partial_v;
  CgState Sst;
  CHK(alloc_state(C, nrhs, Sst));
  // direction ring (batched x update): ring_slots slots if given, else the
  // most slots R in {16, 8, 4} that divide the poll period and fit a quarter
  // of the device memory not otherwise in use (the ring this context already
  // holds counts as free); else (or ring_slots = -1) the fused per-step update
  Ring ring_store;
  const Ring* ring = nullptr;
  int last_it = 0;  // iterations of the previous pass (its last direction sits in slot last_it mod R)
  if (prm->ring_slots >= 0) {
    size_t avail = 0;
    if (C->arena) {  // what the scratch array has left
      avail = C->arena->cap - std::min(C->arena->cap, C->arena->used + 512 + sizeof(double) * 16 * nrhs);
    } else {
      size_t free_b = 0, total_b = 0;
      HIPCHK(hipMemGetInfo(&free_b, &total_b));
      const auto held = C->pool.find("pring");
      avail = (free_b + (held != C->pool.end() ? held->second.n : 0)) / 4;
    }
    for (int R : {16, 8, 4}) {
      const size_t ring_bytes = (size_t)R * bS;
      if (prm->ring_slots > 0 ? R != prm->ring_slots : (check % R != 0 || ring_bytes > avail)) continue;
      void *rb, *ah;
      CHK(ws(C, "pring", ring_bytes, &rb));
      CHK(ws(C, "ahist", sizeof(double) * R * nrhs, &ah));
      ring_store.base = (char*)rb;
      ring_store.slot = bS;
      ring_store.ahist = (double*)ah;
      ring_store.R = R;
      ring_store.F = R / 2;
      ring = &ring_store;
      break;
    }
  }

  // b = g5 R5 phi, |b|^2
  launch_pack(P64, g, phi, be, 0, nrhs, 1, st);
  launch_pack(P64, g, phi, bo, 1, nrhs, 1, st);
  HIPCHK(hipGetLastError());
  std::vector<double> ne, no, bb(nrhs);
  CHK(norms(C, P64, be, nrhs, partial, Sst, ne, st));
  CHK(norms(C, P64, bo, nrhs, partial, Sst, no, st));
  std::vector<int> done(nrhs, 0), iters(nrhs, 0), outers(nrhs, 0), status(nrhs, EOFA_OK);
  for (int r = 0; r < nrhs; ++r) {
    bb[r] = ne[r] + no[r];
    if (!std::isfinite(bb[r])) {  // NaN / Inf in phi: nothing to iterate on
      status[r] = EOFA_ERR_BREAKDOWN;
      done[r] = 1;
    }
  }

  // Schur source b~_o = b_o - Dhop D~ M_ee^-1 b_e (dense: b_o - Dhop D_ee^-1 b_e)
  launch_smat(P64, g, be, te, mats_of(C), F.inv, nrhs, st);
  {
    HopArgs a = base_args(C, P64, 1, nrhs);
    a.in = te;
    a.z = bo;
    a.out = bt;
    CHK(hop(C, P64, F.src, a, st));
  }
  if (prm->use_guess && F.cayley) {
    // x_o = (D~^-1 psi)_o: the right-preconditioned unknown of the guess
    launch_pack(P64, g, psi, tmp, 1, nrhs, 0, st);
    launch_smat(P64, g, tmp, x, mats_of(C), MAT_DT_INV, nrhs, st);
  } else if (prm->use_guess) {
    launch_pack(P64, g, psi, x, 1, nrhs, 0, st);
  } else {
    launch_zero(P64, g, x, nrhs, st);
  }

  std::vector<double> rro, rro_prev(nrhs, 0.0);
  std::vector<int> diverged(nrhs, 0);
  std::vector<int> hbuf(4 * nrhs);
  std::vector<double> hd(2 * nrhs);
  double hop_ms[4] = {0, 0, 0, 0};
  int timed = 0;
  const int max_timed = 256;  // timed iterations per solve (every 8th iteration)
  if (prm->profile && !C->arena && C->events.empty()) {
    C->events.resize(8 * max_timed);
    for (auto& ev : C->events) HIPCHK(hipEventCreate(&ev));
  }

  HopArgs k1 = base_args(C, S, 0, nrhs);
  k1.in = pS;
  k1.out = tS;
  k1.matA = F.m1;
  k1.halt = Sst.halt;
  HopArgs k2 = base_args(C, S, 1, nrhs);
  k2.in = tS;
  k2.y = pS;
  k2.out = wS;
  k2.matB = F.m2;
  k2.partial = partial;
  k2.halt = Sst.halt;
  HopArgs k3 = base_args(C, S, 0, nrhs);
  k3.in = wS;
  k3.out = tS;
  k3.matA = F.m3;
  k3.halt = Sst.halt;
  HopArgs k4 = base_args(C, S, 1, nrhs);
  k4.in = tS;
  k4.y = wS;
  k4.r = rin;
  k4.matA = F.m4a;
  k4.matB = F.m4b;
  k4.alpha = Sst.alpha;
  k4.partial = partial;
  k4.halt = Sst.halt;
  if (prm->rhs_block <= 0 && prm->waves <= 0 && !C->arena) {
    CHK(autotune(C, F, S, nrhs, k1, k2, k3, k4, st));
    const auto pick = C->tuned[tune_key(F, S, nrhs)];
    for (HopArgs* x : {&k1, &k2, &k3, &k4}) {
      x->W = pick.first;
      x->rhs_block = pick.second;
    }
  }

  for (int outer = 0; outer < max_outer; ++outer) {
    // r_o = b~ - M^ x  (FP64)
    if (outer == 0 && !prm->use_guess) {
      launch_convert(P64, P64, g, bt, ro, nrhs, st);
      CHK(norms(C, P64, ro, nrhs, partial, Sst, rro, st));
    } else {
      HopArgs a1 = base_args(C, P64, 0, nrhs);
      a1.in = x;
      a1.out = te;
      a1.matA = F.m1;
      CHK(hop(C, P64, F.k1x, a1, st));
      HopArgs a2 = base_args(C, P64, 1, nrhs);
      a2.in = te;
      a2.y = x;
      a2.z = bt;
      a2.out = ro;
      a2.matB = F.m2;
      a2.partial = partial;
      int nb = 0;
      CHK(hop(C, P64, F.res, a2, st, &nb));
      launch_finalize(FIN_NORM, partial, nb, nrhs, Sst, Sst.norm, st);
      rro.resize(nrhs);
      CHK(fetch(C, Sst.norm, nrhs * sizeof(double), rro.data(), st));
    }
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
      if (done[r]) continue;
      const double res = bb[r] > 0 ? std::sqrt(rro[r] / bb[r]) : (rro[r] == 0.0 ? 0.0 : INFINITY);
      if (!std::isfinite(res)) {
        status[r] = EOFA_ERR_BREAKDOWN;
        done[r] = 1;
        continue;
      }
      if (!fixed && res <= (tolr ? tolr[r] : prm->tol)) done[r] = 1;
      if (!fixed && iters[r] >= prm->max_iter) done[r] = 1;
      if (!done[r]) all = false;
    }
    if (all) break;
    if (fixed && outer >= 1) break;

    // Reliable updates keep the previous pass's direction unless that pass
    // diverged (stopped by its guard) or cut the FP64 residual by less than
    // 2x: then every right-hand side restarts from p = r (kept directions go
    // stale on ill-conditioned systems, where a pass is long in FP16).
    bool restart = !(keep && outer > 0);
    for (int r = 0; r < nrhs && !restart; ++r)
      if (!done[r] && (diverged[r] || rro[r] > 0.25 * rro_prev[r])) restart = true;
    for (int r = 0; r < nrhs; ++r) rro_prev[r] = rro[r];

    // inner CGNR in precision S on M^ e = r_o
    std::vector<int> mi(nrhs);
    std::vector<double> t2(nrhs), gd(nrhs);
    for (int r = 0; r < nrhs; ++r) {
      mi[r] = done[r] ? 0 : (fixed ? prm->fixed_iters : std::max(0, prm->max_iter - iters[r]));
      double it_r = 0.0;
      if (!fixed && !done[r]) {
        const double need = 0.3 * (tolr ? tolr[r] : prm->tol) * std::sqrt(bb[r] / std::max(rro[r], 1e-300));
        it_r = std::min(0.5, std::max(inner_floor, need));
      }
      t2[r] = it_r * it_r;
      // a kept direction may diverge: stop its pass once |r|^2 grows 1e4x
      gd[r] = restart ? 0.0 : 1e4;
      if (!done[r]) outers[r] += 1;
    }
    CHK(put(C, Sst.max_iter, mi.data(), nrhs * sizeof(int), st));
    CHK(put(C, Sst.tol2, t2.data(), nrhs * sizeof(double), st));
    CHK(put(C, Sst.guard, gd.data(), nrhs * sizeof(double), st));
    launch_convert(P64, S, g, ro, rS, nrhs, st);
    {
      HopArgs a3 = base_args(C, S, 0, nrhs);
      a3.in = rS;
      a3.out = tS;
      a3.matA = F.m3;
      CHK(hop(C, S, F.k3, a3, st));
      HopArgs a4 = base_args(C, S, 1, nrhs);
      a4.in = tS;
      a4.y = rS;
      a4.r = rin;
      a4.matA = F.m4a;
      a4.matB = F.m4b;
      a4.partial = partial;
      int nb = 0;
      CHK(hop(C, S, F.k4s, a4, st, &nb));
      launch_finalize(FIN_INIT, partial, nb, nrhs, Sst, nullptr, st);
    }
    // p = r starts the inner CG afresh; a reliable update (keep_direction,
    // after the first pass) keeps the previous pass's direction p, which
    // stays conjugate to within the inner precision, and replaces only r
    void* p0 = ring ? ring->at(0) : pS;
    if (restart && F.ptilde) {  // p~ = D~ r
      launch_smat(S, g, rin, p0, mats_of(C), MAT_DT, nrhs, st);
    } else if (restart) {
      launch_convert(S, S, g, rin, p0, nrhs, st);
    } else if (ring && last_it % ring->R != 0) {  // the kept direction into slot 0
      HIPCHK(hipMemcpyAsync(p0, ring->at(last_it), bS, hipMemcpyDeviceToDevice, st));
    }
    launch_zero(PX, g, xin, nrhs, st);

    if (prm->rhs_block > 0 || prm->waves > 0) {
      const int w = prm->waves > 0 ? prm->waves : default_waves(g.Ls);
      const int rb = prm->rhs_block > 0 ? std::min(prm->rhs_block, nrhs) : nrhs;
      for (HopArgs* x : {&k1, &k2, &k3, &k4}) {
        x->W = w;
        x->rhs_block = rb;
      }
    }
    const int nbh = hop_blocks(S, g.Vh, g.Ls, k1.W);

    int it = 0;
    const int cap = fixed ? prm->fixed_iters : prm->max_iter + 1;
    if (prm->use_graph) {
      // capture check_every iterations once per pass on a non-blocking stream
      // ordered after the caller's stream, then replay; converged right-hand
      // sides are skipped inside the kernels through their halt flags
      if (!C->cap_stream) HIPCHK(hipStreamCreateWithFlags(&C->cap_stream, hipStreamNonBlocking));
      hipStream_t cs = C->cap_stream;
      hipEvent_t join;
      HIPCHK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
      HIPCHK(hipEventRecord(join, st));
      HIPCHK(hipStreamWaitEvent(cs, join, 0));
      hipGraph_t graph;
      hipGraphExec_t exec;
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < check; ++k) {
        const int rc =
            inner_iteration(C, F, S, k1, k2, k3, k4, nbh, nrhs, Sst, partial, xin, rin, pS, cs, nullptr, ring, k);
        if (rc != EOFA_OK) {
          hipGraph_t dead;
          (void)hipStreamEndCapture(cs, &dead);
          if (dead) (void)hipGraphDestroy(dead);
          return rc;
        }
      }
      HIPCHK(hipStreamEndCapture(cs, &graph));
      HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      while (true) {
        HIPCHK(hipGraphLaunch(exec, cs));
        it += check;
        HIPCHK(hipMemcpyAsync(C->host_stage, Sst.halt, nrhs * sizeof(int), hipMemcpyDeviceToHost, cs));
        HIPCHK(hipStreamSynchronize(cs));
        std::memcpy(hbuf.data(), C->host_stage, nrhs * sizeof(int));
        bool stop = true;
        for (int r = 0; r < nrhs; ++r) stop = stop && hbuf[r] != 0;
        if (stop || it >= cap) break;
      }
      HIPCHK(hipGraphExecDestroy(exec));
      HIPCHK(hipGraphDestroy(graph));
      HIPCHK(hipEventRecord(join, cs));
      HIPCHK(hipStreamWaitEvent(st, join, 0));
      HIPCHK(hipEventDestroy(join));
    } else {
      while (true) {
        // timed iterations sit between host polls (which drain the queue), so the
        // events bracket the kernels and not host launch latency (a
        // no-allocation call creates no events and times nothing)
        const bool prof = prm->profile && !C->arena && timed < max_timed && (it % 8 == 4);
        hipEvent_t* ev = prof ? &C->events[timed * 8] : nullptr;
        CHK(inner_iteration(C, F, S, k1, k2, k3, k4, nbh, nrhs, Sst, partial, xin, rin, pS, st, ev, ring, it));
        if (prof) ++timed;
        ++it;
        if (it % check == 0 || it >= cap) {
          CHK(fetch(C, Sst.halt, nrhs * sizeof(int), hbuf.data(), st));
          bool stop = true;
          for (int r = 0; r < nrhs; ++r) stop = stop && hbuf[r] != 0;
          if (stop || it >= cap) break;
        }
      }
    }
    if (ring && it % ring->F != 0) {  // the steps since the last batched x update
      const int rem = it % ring->F;
      launch_x_flush(S, g, xin, ring->base, ring->slot, (it - rem) % ring->R, rem, ring->R, ring->ahist, nrhs, st);
    }
    last_it = it;
    HIPCHK(hipGetLastError());
    std::vector<int> hi(nrhs), hb(nrhs);
    CHK(fetch(C, Sst.iter, nrhs * sizeof(int), hi.data(), st));
    CHK(fetch(C, Sst.breakdown, nrhs * sizeof(int), hb.data(), st));
    const size_t bX1 = packed_bytes(PX, g, 1);
    for (int r = 0; r < nrhs; ++r) {
      diverged[r] = 0;
      if (done[r]) continue;
      iters[r] += hi[r];
      if (hb[r] == 2) {  // a diverged pass contributes nothing; the next one restarts
        diverged[r] = 1;
        HIPCHK(hipMemsetAsync((char*)xin + bX1 * r, 0, bX1, st));
      } else if (hb[r]) {
        status[r] = EOFA_ERR_BREAKDOWN;
        done[r] = 1;
      }
    }
    if (F.ptilde) {  // the pass accumulated x~ = D~ e: x += D~^-1 x~ (tmp is free here)
      launch_smat(PX, g, xin, tmp, mats_of(C), MAT_DT_INV, nrhs, st);
      launch_axpy_to64(PX, g, x, tmp, nrhs, st);
    } else {
      launch_axpy_to64(PX, g, x, xin, nrhs, st);
    }
  }

  std::vector<double> re, rodd;
  CHK(reconstruct(C, F, nrhs, x, be, bo, te, tmp, ro, partial, Sst, psi, re, rodd, st));
  const double t1 = now_s();
  for (int j = 0; j < timed; ++j) {  // events are read only after the solve: no mid-solve host stalls
    float ms;
    for (int k = 0; k < 4; ++k) {
      HIPCHK(hipEventElapsedTime(&ms, C->events[j * 8 + 2 * k], C->events[j * 8 + 2 * k + 1]));
      hop_ms[k] += ms;
    }
  }

  int worst = EOFA_OK;
  for (int r = 0; r < nrhs; ++r) {
    const double tr = bb[r] > 0 ? std::sqrt((re[r] + rodd[r]) / bb[r]) : ((re[r] + rodd[r]) == 0.0 ? 0.0 : NAN);
    const bool conv = std::isfinite(tr) && tr <= (tolr ? tolr[r] : prm->tol);
    if (status[r] == EOFA_OK && !conv && !fixed) status[r] = std::isfinite(tr) ? EOFA_ERR_NOT_CONVERGED : EOFA_ERR_BREAKDOWN;
    if (stats) {
      eofa_solver_stats& o = stats[r];
      std::memset(&o, 0, sizeof(o));
      o.iters = iters[r];
      o.outer_iters = outers[r];
      o.converged = conv ? 1 : 0;
      o.status = status[r];
      o.true_resid = tr;
      o.seconds = t1 - t0;
      for (int k = 0; k < 4; ++k) o.hop_ms[k] = hop_ms[k];
      o.hop_timed = timed;
      o.waves = k1.W;
      o.rhs_block = k1.rhs_block;
    }
    if (status[r] != EOFA_OK && (worst == EOFA_OK || status[r] == EOFA_ERR_BREAKDOWN)) worst = status[r];
  }
  if (worst == EOFA_ERR_NOT_CONVERGED) g_err = "solve did not reach the requested true residual";
  if (worst == EOFA_ERR_BREAKDOWN) g_err = "CG breakdown (non-finite value or non-positive curvature)";
  return worst;
}

int check_params(const eofa_solver_params* prm) {
  if (!prm) return fail(EOFA_ERR_INVALID, "params is NULL");
  CHK(check_prec(prm->inner_prec));
  if (prm->fixed_iters <= 0 && !(prm->tol > 0.0)) return fail(EOFA_ERR_INVALID, "tol must be > 0");
  if (prm->fixed_iters <= 0 && prm->max_iter < 1) return fail(EOFA_ERR_INVALID, "max_iter must be >= 1");
  if (prm->precond != 0 && prm->precond != 1) return fail(EOFA_ERR_INVALID, "precond must be 0 or 1");
  if (prm->precond == 1 && prm->fixed_iters > 0)
    return fail(EOFA_ERR_INVALID, "fixed_iters applies to CGNR only (precond = 0)");
  if (prm->form != 0 && prm->form != 1) return fail(EOFA_ERR_INVALID, "form must be 0 or 1");
  if (prm->form == 1 && prm->precond != 0)
    return fail(EOFA_ERR_INVALID, "the dense form (form = 1) is solved by CGNR only (precond = 0)");
  if (prm->waves != 0 && prm->waves != 1 && prm->waves != 2 && prm->waves != 4)
    return fail(EOFA_ERR_INVALID, "waves must be 0 (autotune), 1, 2 or 4");
  if (prm->rhs_block < 0) return fail(EOFA_ERR_INVALID, "rhs_block must be >= 0");
  const int rs = prm->ring_slots, chk = prm->check_every > 0 ? prm->check_every : 16;
  if (rs != -1 && rs != 0 && rs != 4 && rs != 8 && rs != 16)
    return fail(EOFA_ERR_INVALID, "ring_slots must be -1, 0, 4, 8 or 16");
  if (rs > 0 && chk % rs != 0) return fail(EOFA_ERR_INVALID, "ring_slots must divide check_every");
  return EOFA_OK;
}

}  // namespace

// A = M^dag M of the odd Schur system of sys on packed FP32 odd half-fields of
// one right-hand side: out = A in, FP32 arithmetic (K1, K2, K3, K4S). The
// network's residual loss uses it; workspace comes from the context pool.
int eofa::normal_op_fp32(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, hipStream_t st) {
  const Geometry& g = C->g;
  CHK(upload_systems(C, sys, 1, st));
  const size_t b32 = packed_bytes(P32, g, 1);
  void *te, *w, *pv;
  CHK(ws(C, "na_te", b32, &te));
  CHK(ws(C, "na_w", b32, &w));
  const int maxblk = std::max(hop_blocks(P32, g.Vh, g.Ls, 1), (g.Ls * g.Vh + 255) / 256);
  CHK(ws(C, "na_partial", sizeof(double) * (size_t)maxblk, &pv));
  HopArgs k1 = base_args(C, P32, 0, 1);
  k1.in = in;
  k1.out = te;
  k1.matA = MAT_MEE_INV;
  CHK(hop(C, P32, ROLE_K1, k1, st));
  HopArgs k2 = base_args(C, P32, 1, 1);
  k2.in = te;
  k2.y = in;
  k2.out = w;
  k2.matB = MAT_MEE;
  k2.partial = (double*)pv;
  CHK(hop(C, P32, ROLE_K2, k2, st));
  HopArgs k3 = base_args(C, P32, 0, 1);
  k3.in = w;
  k3.out = te;
  k3.matA = MAT_MEE_INV_T;
  CHK(hop(C, P32, ROLE_K3, k3, st));
  HopArgs k4 = base_args(C, P32, 1, 1);
  k4.in = te;
  k4.y = w;
  k4.r = out;
  k4.matA = MAT_NEG_DT_T;
  k4.matB = MAT_MEE_T;
  k4.partial = (double*)pv;
  CHK(hop(C, P32, ROLE_K4S, k4, st));
  return EOFA_OK;
}

// ---------------------------------------------------------------------------
// flexible CG on the normal equations (learned preconditioner) and the
// training-pair generator

namespace {

// Device scalars of the flexible-CG recurrence (doubles), then one int flag.
// FG_WWS + j: <p_j, A p_j> of window slot j.
constexpr int FG_MAXW = 32;  // most previous directions kept
enum FgScalar { FG_WW = 0, FG_QZ = 2, FG_PR = 4, FG_ALPHA = 6, FG_BETA = 8, FG_NRM = 10, FG_WWS = 12,
                FG_BETAS = FG_WWS + FG_MAXW + 2, FG_N = FG_BETAS + 2 * FG_CHUNK };

// One right-hand side, FP64 throughout, on the odd Schur system:
//   s = b~ - M^ x (Schur residual), r = M^dag s (normal residual),
//   z = N(r); p = z - sum_j (<A p_j, z>/<p_j, A p_j>) p_j over the last m
//   directions; w = M^ p; q = M^dag w; alpha = <p, r>/|w|^2;
//   x += alpha p; r -= alpha q; s -= alpha w
// (Notay's flexible CG, A = M^dag M, truncated to m previous directions;
// m = 1 is the one-term recurrence, which for N = 1 is CG).
struct Fgcg {
  eofa_ctx* C = nullptr;
  hipStream_t st = nullptr;
  void *be, *bo, *bt, *x, *s, *r, *p, *q, *w, *z, *te, *tmp, *r32, *z32;
  std::vector<void*> ps, qs;  // window slots (m >= 2)
  int m = 1, nvalid = 0, cur = 0;
  double* partial = nullptr;
  double* sc = nullptr;
  int* bad = nullptr;
  CgState Sst;
  int n = 0;  // complex numbers in one FP64 odd half-field
  double bb = 0.0;
  bool first = true;

  int set_window(int mw) {
    m = std::max(1, std::min(mw, FG_MAXW));
    if (m == 1) return EOFA_OK;
    const size_t b64 = packed_bytes(P64, C->g, 1);
    ps.assign(m + 1, nullptr);
    qs.assign(m + 1, nullptr);
    for (int j = 0; j <= m; ++j) {
      CHK(ws(C, ("fg_wp" + std::to_string(j)).c_str(), b64, &ps[j]));
      CHK(ws(C, ("fg_wq" + std::to_string(j)).c_str(), b64, &qs[j]));
    }
    return EOFA_OK;
  }

  int init(const eofa_system* sys, const void* phi) {
    const Geometry& g = C->g;
    CHK(upload_systems(C, sys, 1, st));
    CHK(stage(C, 1024));
    const size_t b64 = packed_bytes(P64, g, 1), b32 = packed_bytes(P32, g, 1);
    const char* names[12] = {"fg_be", "fg_bo", "fg_bt", "fg_x", "fg_s", "fg_r",
                             "fg_p", "fg_q", "fg_w", "fg_z", "fg_te", "fg_tmp"};
    void** bufs[12] = {&be, &bo, &bt, &x, &s, &r, &p, &q, &w, &z, &te, &tmp};
    for (int k = 0; k < 12; ++k) CHK(ws(C, names[k], b64, bufs[k]));
    CHK(ws(C, "fg_r32", b32, &r32));
    CHK(ws(C, "fg_z32", b32, &z32));
    const int maxblk = std::max({hop_blocks(P64, g.Vh, g.Ls, 1), (g.Ls * g.Vh + 255) / 256, 512 * FG_CHUNK});
    void* pv;
    CHK(ws(C, "fg_partial", sizeof(double) * 2 * (size_t)maxblk, &pv));
    partial = (double*)pv;
    void* sv;
    CHK(ws(C, "fg_scalars", sizeof(double) * FG_N + 64, &sv));
    sc = (double*)sv;
    bad = (int*)(sc + FG_N);
    CHK(alloc_state(C, 1, Sst));
    n = (int)(b64 / 16);
    HIPCHK(hipMemsetAsync(sv, 0, sizeof(double) * FG_N + 64, st));
    launch_pack(P64, g, phi, be, 0, 1, 1, st);
    launch_pack(P64, g, phi, bo, 1, 1, 1, st);
    HIPCHK(hipGetLastError());
    std::vector<double> ne, no;
    CHK(norms(C, P64, be, 1, partial, Sst, ne, st));
    CHK(norms(C, P64, bo, 1, partial, Sst, no, st));
    bb = ne[0] + no[0];
    launch_smat(P64, g, be, te, mats_of(C), MAT_MEE_INV, 1, st);
    HopArgs a = base_args(C, P64, 1, 1);
    a.in = te;
    a.z = bo;
    a.out = bt;
    CHK(hop(C, P64, ROLE_SRC, a, st));
    launch_zero(P64, g, x, 1, st);
    launch_convert(P64, P64, g, bt, s, 1, st);
    return normal_residual();
  }

  // r = M^dag s, |r|^2 -> sc[FG_NRM]; the next iteration starts a new recurrence
  int normal_residual() {
    HopArgs a3 = base_args(C, P64, 0, 1);
    a3.in = s;
    a3.out = te;
    a3.matA = MAT_MEE_INV_T;
    CHK(hop(C, P64, ROLE_K3, a3, st));
    HopArgs a4 = base_args(C, P64, 1, 1);
    a4.in = te;
    a4.y = s;
    a4.r = r;
    a4.matA = MAT_NEG_DT_T;
    a4.matB = MAT_MEE_T;
    a4.partial = partial;
    int nb = 0;
    CHK(hop(C, P64, ROLE_K4S, a4, st, &nb));
    launch_finalize(FIN_NORM, partial, nb, 1, Sst, sc + FG_NRM, st);
    first = true;
    nvalid = 0;
    return EOFA_OK;
  }

  // s = b~ - M^ x recomputed in FP64; returns |s|^2 on the host
  int true_schur(double* out) {
    HopArgs a1 = base_args(C, P64, 0, 1);
    a1.in = x;
    a1.out = te;
    a1.matA = MAT_MEE_INV;
    CHK(hop(C, P64, ROLE_K1, a1, st));
    HopArgs a2 = base_args(C, P64, 1, 1);
    a2.in = te;
    a2.y = x;
    a2.z = bt;
    a2.out = s;
    a2.matB = MAT_MEE;
    a2.partial = partial;
    int nb = 0;
    CHK(hop(C, P64, ROLE_RES, a2, st, &nb));
    launch_finalize(FIN_NORM, partial, nb, 1, Sst, sc + FG_NRM + 1, st);
    return fetch(C, sc + FG_NRM + 1, sizeof(double), out, st);
  }

  int iterate(eofa_net* net) {
    const Geometry& g = C->g;
    if (net) {
      launch_convert(P64, P32, g, r, r32, 1, st);
      CHK(net_apply_internal(C, net, r32, z32, st));
      launch_convert(P32, P64, g, z32, z, 1, st);
    } else {
      launch_convert(P64, P64, g, r, z, 1, st);
    }
    double* ww = sc + FG_WW;
    if (m == 1) {
      if (first) {
        launch_convert(P64, P64, g, z, p, 1, st);
      } else {
        launch_cdot(n, q, z, partial, sc + FG_QZ, st);
        launch_fgcg_ratio(sc + FG_QZ, sc + FG_WW, -1.0, sc + FG_BETA, bad, st);
        launch_cxpby_dev(n, z, sc + FG_BETA, p, st);
      }
    } else {
      // new direction in slot cur, A-orthogonal to the previous nvalid ones
      // (classical Gram-Schmidt: every coefficient from z)
      if (first) nvalid = 0;
      p = ps[cur];
      q = qs[cur];
      ww = sc + FG_WWS + cur;
      // (up to FG_CHUNK directions per pass over z and per pass over p)
      launch_convert(P64, P64, g, z, p, 1, st);
      for (int k0 = 1; k0 <= nvalid; k0 += FG_CHUNK) {
        const int nq = std::min(FG_CHUNK, nvalid - k0 + 1);
        FgPtrs qv{}, pv{};
        for (int t = 0; t < nq; ++t) {
          const int j = (cur - (k0 + t) + m + 1) % (m + 1);
          qv.v[t] = qs[j];
          qv.ww[t] = sc + FG_WWS + j;
          pv.v[t] = ps[j];
        }
        launch_fgcg_orth_coefs(n, nq, qv, z, partial, sc + FG_BETAS, bad, st);
        launch_caxpy_multi(n, nq, pv, sc + FG_BETAS, p, st);
      }
    }
    first = false;
    HopArgs k1 = base_args(C, P64, 0, 1);
    k1.in = p;
    k1.out = te;
    k1.matA = MAT_MEE_INV;
    CHK(hop(C, P64, ROLE_K1, k1, st));
    HopArgs k2 = base_args(C, P64, 1, 1);
    k2.in = te;
    k2.y = p;
    k2.out = w;
    k2.matB = MAT_MEE;
    k2.partial = partial;
    int nb = 0;
    CHK(hop(C, P64, ROLE_K2, k2, st, &nb));
    launch_finalize(FIN_NORM, partial, nb, 1, Sst, ww, st);
    HopArgs k3 = base_args(C, P64, 0, 1);
    k3.in = w;
    k3.out = te;
    k3.matA = MAT_MEE_INV_T;
    CHK(hop(C, P64, ROLE_K3, k3, st));
    HopArgs k4 = base_args(C, P64, 1, 1);
    k4.in = te;
    k4.y = w;
    k4.r = q;
    k4.matA = MAT_NEG_DT_T;
    k4.matB = MAT_MEE_T;
    k4.partial = partial;
    CHK(hop(C, P64, ROLE_K4S, k4, st, &nb));
    launch_cdot(n, p, r, partial, sc + FG_PR, st);
    launch_fgcg_ratio(sc + FG_PR, ww, 1.0, sc + FG_ALPHA, bad, st);
    nb = launch_fgcg_update(n, sc + FG_ALPHA, x, r, s, p, q, w, partial, st);
    launch_finalize(FIN_NORM, partial, nb, 2, Sst, sc + FG_NRM, st);
    if (m > 1) {
      nvalid = std::min(nvalid + 1, m);
      cur = (cur + 1) % (m + 1);
    }
    HIPCHK(hipGetLastError());
    return EOFA_OK;
  }

  // host read of |r|^2, |s|^2 and the breakdown flag
  int poll(double* rr, double* ss, int* flag) {
    double h[FG_N + 2];
    CHK(fetch(C, sc, sizeof(double) * FG_N + sizeof(int), h, st));
    *rr = h[FG_NRM];
    *ss = h[FG_NRM + 1];
    std::memcpy(flag, h + FG_N, sizeof(int));
    return EOFA_OK;
  }
};

int fgcg_one(eofa_ctx* C, const eofa_system* sys, const void* phi, void* psi, const eofa_solver_params* prm,
             eofa_solver_stats* out, hipStream_t st) {
  const double t0 = now_s();
  eofa_net* net = const_cast<eofa_net*>(prm->net);
  Fgcg F;
  F.C = C;
  F.st = st;
  CHK(F.init(sys, phi));
  CHK(F.set_window(prm->fcg_window > 0 ? prm->fcg_window : 1));
  bool guess_done = false;
  if (prm->use_guess && std::isfinite(F.bb)) {
    // start from x_o = (D~^-1 psi)_o: s = b~ - M^ x, r = M^dag s
    launch_pack(P64, C->g, psi, F.tmp, 1, 1, 0, st);
    launch_smat(P64, C->g, F.tmp, F.x, mats_of(C), MAT_DT_INV, 1, st);
    double s2;
    CHK(F.true_schur(&s2));
    CHK(F.normal_residual());
    guess_done = F.bb > 0.0 && std::sqrt(s2 / F.bb) <= prm->tol;
  }
  const int check = prm->check_every > 0 ? prm->check_every : 16;
  const int max_restart = std::max(1, prm->max_outer);
  const int stall = std::max(256, 16 * check);  // iterations without a 0.7x gain in |s| before falling back
  int status = EOFA_OK, it = 0, restarts = 0;
  bool fallback = !std::isfinite(F.bb);
  bool converged = false;
  double best = INFINITY;
  int best_it = 0;
  if (F.bb == 0.0 || guess_done) converged = true;
  while (!fallback && !converged) {
    CHK(F.iterate(net));
    ++it;
    if (it % check != 0 && it < prm->max_iter) continue;
    double rr, ss;
    int flag;
    CHK(F.poll(&rr, &ss, &flag));
    const double res = std::sqrt(ss / F.bb);
    if (flag || !std::isfinite(res) || !std::isfinite(rr)) {
      fallback = true;
      break;
    }
    if (res < 0.7 * best) {
      best = res;
      best_it = it;
    }
    if (res <= 0.5 * prm->tol || it >= prm->max_iter) {
      double st2;
      CHK(F.true_schur(&st2));
      const double tres = std::sqrt(st2 / F.bb);
      if (tres <= prm->tol) {
        converged = true;
        break;
      }
      if (it >= prm->max_iter) {
        status = EOFA_ERR_NOT_CONVERGED;
        break;
      }
      if (++restarts >= max_restart) {
        fallback = true;
        break;
      }
      CHK(F.normal_residual());  // restart from the true residual
      best = tres;
      best_it = it;
      continue;
    }
    if (it - best_it >= stall) fallback = true;
  }
  if (fallback) {
    eofa_solver_params p2 = *prm;
    p2.precond = 0;
    p2.net = nullptr;
    p2.max_iter = std::max(1, prm->max_iter - it);
    const int rc = solve_batch(C, sys, 1, phi, psi, &p2, out, st);
    if (out) {
      out->fell_back = 1;
      out->iters += it;
      out->seconds = now_s() - t0;
    }
    return rc;
  }
  std::vector<double> re, rodd;
  CHK(reconstruct(C, kCayley, 1, F.x, F.be, F.bo, F.te, F.tmp, F.s, F.partial, F.Sst, psi, re, rodd, st));
  const double tr = F.bb > 0 ? std::sqrt((re[0] + rodd[0]) / F.bb) : ((re[0] + rodd[0]) == 0.0 ? 0.0 : NAN);
  const bool conv = std::isfinite(tr) && tr <= prm->tol;
  if (status == EOFA_OK && !conv) status = std::isfinite(tr) ? EOFA_ERR_NOT_CONVERGED : EOFA_ERR_BREAKDOWN;
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->iters = it;
    out->outer_iters = restarts + 1;
    out->converged = conv ? 1 : 0;
    out->status = status;
    out->true_resid = tr;
    out->seconds = now_s() - t0;
  }
  if (status == EOFA_ERR_NOT_CONVERGED) g_err = "flexible CG did not reach the requested true residual";
  if (status == EOFA_ERR_BREAKDOWN) g_err = "flexible CG breakdown (non-finite residual)";
  return status;
}

}  // namespace

extern "C" int eofa_cg_pairs(eofa_ctx* C, const eofa_system* sys, const void* phi, int32_t npairs, int32_t first,
                             int32_t stride, double tol, int32_t max_iter, void* r_out, void* e_out,
                             int32_t* recorded, int32_t* iters, void* stream) {
  if (!C || !phi || !r_out || !e_out || !recorded) return fail(EOFA_ERR_INVALID, "eofa_cg_pairs: NULL argument");
  if (npairs < 1 || first < 0 || stride < 1 || !(tol > 0.0) || max_iter < 1)
    return fail(EOFA_ERR_INVALID, "eofa_cg_pairs: need npairs >= 1, first >= 0, stride >= 1, tol > 0, max_iter >= 1");
  CHK(check_systems(sys, 1));
  hipStream_t st = (hipStream_t)stream;
  const Geometry& g = C->g;
  Fgcg F;
  F.C = C;
  F.st = st;
  CHK(F.init(sys, phi));
  if (!std::isfinite(F.bb)) return fail(EOFA_ERR_BREAKDOWN, "eofa_cg_pairs: non-finite source");
  const size_t b64 = packed_bytes(P64, g, 1), b32 = packed_bytes(P32, g, 1);
  void* xs = nullptr;
  if (hipMalloc(&xs, b64 * (size_t)npairs) != hipSuccess) {
    (void)hipGetLastError();
    return fail(EOFA_ERR_OOM, "eofa_cg_pairs: hipMalloc failed for the stored iterates");
  }
  auto run = [&]() -> int {
    double rr0, ss, rr;
    int flag;
    CHK(F.poll(&rr0, &ss, &flag));
    int j = 0, it = 0;
    const int check = 16;
    while (true) {
      if (j < npairs && it == first + j * stride) {
        launch_convert(P64, P32, g, F.r, (char*)r_out + b32 * j, 1, st);
        launch_convert(P64, P64, g, F.x, (char*)xs + b64 * j, 1, st);
        ++j;
      }
      if (it >= max_iter) {
        *recorded = j;
        if (iters) *iters = it;
        return fail(EOFA_ERR_NOT_CONVERGED, "eofa_cg_pairs: CG did not reach tol within max_iter");
      }
      CHK(F.iterate(nullptr));
      ++it;
      if (it % check == 0) {
        CHK(F.poll(&rr, &ss, &flag));
        if (flag || !std::isfinite(rr)) return fail(EOFA_ERR_BREAKDOWN, "eofa_cg_pairs: CG breakdown");
        if (rr <= tol * tol * rr0) break;
      }
    }
    // e_j = x* - x_j in FP64, stored in FP32
    for (int k = 0; k < j; ++k) {
      launch_convert(P64, P64, g, F.x, F.tmp, 1, st);
      launch_caxpy(F.n, -1.0, 0.0, (char*)xs + b64 * k, F.tmp, st);
      launch_convert(P64, P32, g, F.tmp, (char*)e_out + b32 * k, 1, st);
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    *recorded = j;
    if (iters) *iters = it;
    return EOFA_OK;
  };
  const int rc = run();
  (void)hipStreamSynchronize(st);
  (void)hipFree(xs);
  return rc;
}

extern "C" int eofa_cg_solve(eofa_ctx* C, const eofa_system* sys, const void* phi, void* psi, int32_t nrhs,
                             const eofa_solver_params* prm, eofa_solver_stats* stats, void* stream) {
  if (!C || !phi || !psi) return fail(EOFA_ERR_INVALID, "eofa_cg_solve: NULL argument");
  if (phi == psi) return fail(EOFA_ERR_INVALID, "eofa_cg_solve: phi and psi alias");
  CHK(check_systems(sys, nrhs));
  CHK(check_params(prm));
  if (prm->precond == 0) return solve_batch(C, sys, nrhs, phi, psi, prm, stats, (hipStream_t)stream);
  const size_t fbytes = (size_t)C->g.Ls * C->g.V * 12 * 16;
  int worst = EOFA_OK;
  for (int k = 0; k < nrhs; ++k) {
    const int rc = fgcg_one(C, sys + k, (const char*)phi + fbytes * k, (char*)psi + fbytes * k, prm,
                            stats ? stats + k : nullptr, (hipStream_t)stream);
    if (rc == EOFA_ERR_INVALID || rc == EOFA_ERR_HIP || rc == EOFA_ERR_OOM) return rc;
    if (rc != EOFA_OK && (worst == EOFA_OK || rc == EOFA_ERR_BREAKDOWN)) worst = rc;
  }
  return worst;
}

extern "C" int eofa_cg_solve_noalloc(eofa_ctx* C, const eofa_system* sys, const void* phi, void* psi,
                                     int32_t nrhs, const eofa_solver_params* prm, eofa_solver_stats* stats,
                                     void* stream) {
  if (!C || !phi || !psi) return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: NULL argument");
  if (phi == psi) return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: phi and psi alias");
  CHK(check_systems(sys, nrhs));
  CHK(check_params(prm));
  if (prm->precond != 0) return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: precond must be 0 (CGNR)");
  if (prm->use_graph) return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: use_graph must be 0");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != C->device) return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: the context's device is not current");
  void* base = scratch_ptr(dev);
  if (!base) return fail(EOFA_ERR_HIP, "eofa_cg_solve_noalloc: scratch address not set up on this device");
  // the solve's buffers (packed fields, partial sums, CG scalars, coefficients),
  // each aligned to 256 bytes; the direction ring is added only if it fits
  const Geometry& g = C->g;
  const int S = prm->inner_prec, PX = S == P64 ? P64 : P32;
  const size_t b64 = packed_bytes(P64, g, nrhs), bS = packed_bytes(S, g, nrhs), bX = packed_bytes(PX, g, nrhs);
  const size_t maxblk = std::max(hop_blocks(P64, g.Vh, g.Ls, 1), (g.Ls * g.Vh + 255) / 256);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t need = 7 * al(b64) + 5 * al(bS) + al(bX) + al(sizeof(double) * maxblk * nrhs) +
                      al((8 * sizeof(double) + 5 * sizeof(int)) * nrhs + 64) +
                      al(sizeof(double) * (mats_per_rhs(g) * nrhs + nrhs + scoef_per_rhs(g) * nrhs));
  if (need > kNoallocBytes)
    return fail(EOFA_ERR_INVALID, "eofa_cg_solve_noalloc: needs " + std::to_string((need + (1 << 20) - 1) >> 20) +
                                      " MiB of workspace for this lattice and nrhs; the scratch array holds " +
                                      std::to_string(kNoallocBytes >> 20) + " MiB");
  Arena A;
  A.base = (char*)base;
  A.cap = kNoallocBytes;
  struct Guard {
    eofa_ctx* C;
    ~Guard() {
      C->arena = nullptr;
      C->mats_active = nullptr;
    }
  } guard{C};
  C->arena = &A;
  eofa_solver_params p2 = *prm;
  p2.profile = 0;
  return solve_batch(C, sys, nrhs, phi, psi, &p2, stats, (hipStream_t)stream);
}

extern "C" int eofa_fifth_matrix(const eofa_action* act, const eofa_system* sys, int32_t mat, double* out) {
  if (!act || !sys || !out) return fail(EOFA_ERR_INVALID, "eofa_fifth_matrix: NULL argument");
  if (mat < 0 || mat >= NMAT) return fail(EOFA_ERR_INVALID, "matrix id out of range");
  if (act->Ls < 2 || act->Ls > 32 || act->Ls % 2 != 0) return fail(EOFA_ERR_INVALID, "Ls must be even, 2..32");
  if (std::fabs(act->b5 - act->c5 - 1.0) > 1e-12) return fail(EOFA_ERR_INVALID, "b5 - c5 must be 1 (d = 1/2)");
  CHK(check_systems(sys, 1));
  Geometry g;
  for (int k = 0; k < 4; ++k) g.L[k] = act->dims[k];
  g.Ls = act->Ls;
  g.V = g.Vh = 0;
  const size_t n = (size_t)g.Ls * g.Ls;
  std::vector<double> all(NMAT * 2 * n);
  std::string err;
  const int rc = build_fifth(g, act->M5, act->b5, act->c5, *sys, all.data(), err);
  if (rc != EOFA_OK) return fail(rc, err);
  std::memcpy(out, all.data() + (size_t)mat * 2 * n, sizeof(double) * 2 * n);
  return EOFA_OK;
}

namespace {

// Small dense complex solve G c = f (Gaussian elimination, partial pivoting);
// false if G is numerically singular.
bool solve_small(int n, std::vector<std::complex<double>> G, std::vector<std::complex<double>>& f) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(G[r * n + c]) > std::abs(G[piv * n + c])) piv = r;
    if (!(std::abs(G[piv * n + c]) > 1e-300) || !std::isfinite(std::abs(G[piv * n + c]))) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(G[c * n + k], G[piv * n + k]);
      std::swap(f[c], f[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const std::complex<double> m = G[r * n + c] / G[c * n + c];
      for (int k = c; k < n; ++k) G[r * n + k] -= m * G[c * n + k];
      f[r] -= m * f[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int k = c + 1; k < n; ++k) f[c] -= G[c * n + k] * f[k];
    f[c] /= G[c * n + c];
  }
  for (auto& v : f)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
  return true;
}

// Chronological forecast of the next pole's solution (Sec. VI B, after
// Brower et al.): guess = sum_k c_k psi_k over the previous solutions psi_k of
// the same side, with sum_k c_k psi_l^dag A psi_k = psi_l^dag rhs for every l,
// A = H(m_op) + beta Delta_chi P_chi of the next pole (the minimiser of
// psi^dag A psi - rhs^dag psi - psi^dag rhs on their span). A psi_k is formed
// in the Cayley form, A psi = g5 R5 M_C D~^-1 psi (App. B.2), M_C on both
// parities by the FULLRES role with a zero source. Fields: canonical FP64.
int forecast(eofa_ctx* C, const eofa_system* sys, const void* rhs, const std::vector<const void*>& prev,
             void* guess, hipStream_t st) {
  const Geometry& g = C->g;
  const int N = (int)prev.size();
  CHK(upload_systems(C, sys, 1, st));
  const size_t b64 = packed_bytes(P64, g, 1);
  const size_t fbytes = (size_t)g.Ls * g.V * 12 * 16;
  void *t, *xe, *xo, *me, *mo, *zero, *g5, *pv, *dv;
  CHK(ws(C, "fc_t", b64, &t));
  CHK(ws(C, "fc_xe", b64, &xe));
  CHK(ws(C, "fc_xo", b64, &xo));
  CHK(ws(C, "fc_me", b64, &me));
  CHK(ws(C, "fc_mo", b64, &mo));
  CHK(ws(C, "fc_zero", b64, &zero));
  CHK(ws(C, "fc_g5", 2 * b64 * (size_t)N, &g5));
  const int maxblk = std::max({hop_blocks(P64, g.Vh, g.Ls, 1), (g.Ls * g.Vh + 255) / 256, 2048});
  CHK(ws(C, "fc_partial", sizeof(double) * 2 * (size_t)maxblk, &pv));
  CHK(ws(C, "fc_dot", sizeof(double) * (4 * (size_t)N * N + 2 * (size_t)N), &dv));
  CHK(stage(C, sizeof(double) * (4 * (size_t)N * N + 2 * (size_t)N)));
  double* partial = (double*)pv;
  double* dots = (double*)dv;  // [l][k][parity][re, im], then f[l][re, im]
  launch_zero(P64, g, zero, 1, st);
  const int nh = (int)(b64 / 16);
  for (int l = 0; l < N; ++l) {
    launch_pack(P64, g, prev[l], (char*)g5 + (2 * l) * b64, 0, 1, 1, st);
    launch_pack(P64, g, prev[l], (char*)g5 + (2 * l + 1) * b64, 1, 1, 1, st);
  }
  for (int k = 0; k < N; ++k) {
    launch_pack(P64, g, prev[k], t, 0, 1, 0, st);
    launch_smat(P64, g, t, xe, mats_of(C), MAT_DT_INV, 1, st);
    launch_pack(P64, g, prev[k], t, 1, 1, 0, st);
    launch_smat(P64, g, t, xo, mats_of(C), MAT_DT_INV, 1, st);
    for (int p = 0; p < 2; ++p) {  // out_p = 0 - (M_ee x_p + Dhop D~ x_{1-p}) = -(M_C D~^-1 psi_k)_p
      HopArgs a = base_args(C, P64, p, 1);
      a.in = p ? xe : xo;
      a.y = p ? xo : xe;
      a.z = zero;
      a.out = p ? mo : me;
      a.matB = MAT_MEE;
      a.partial = partial;
      CHK(hop(C, P64, ROLE_FULLRES, a, st));
    }
    for (int l = 0; l < N; ++l) {
      launch_cdot(nh, (char*)g5 + (2 * l) * b64, me, partial, dots + 4 * (l * N + k), st);
      launch_cdot(nh, (char*)g5 + (2 * l + 1) * b64, mo, partial, dots + 4 * (l * N + k) + 2, st);
    }
  }
  const int nfull = (int)(fbytes / 16);
  for (int l = 0; l < N; ++l) launch_cdot(nfull, prev[l], rhs, partial, dots + 4 * N * N + 2 * l, st);
  HIPCHK(hipGetLastError());
  std::vector<double> h(4 * (size_t)N * N + 2 * (size_t)N);
  CHK(fetch(C, dots, sizeof(double) * h.size(), h.data(), st));
  std::vector<std::complex<double>> G((size_t)N * N), f(N);
  for (int l = 0; l < N; ++l) {
    for (int k = 0; k < N; ++k) {
      const double* d = h.data() + 4 * (l * N + k);
      G[l * N + k] = -std::complex<double>(d[0] + d[2], d[1] + d[3]);
    }
    f[l] = {h[4 * N * N + 2 * l], h[4 * N * N + 2 * l + 1]};
  }
  HIPCHK(hipMemsetAsync(guess, 0, fbytes, st));
  if (!solve_small(N, G, f)) return EOFA_OK;  // no usable forecast: start from zero
  for (int k = 0; k < N; ++k) launch_caxpy(nfull, f[k].real(), f[k].imag(), prev[k], guess, st);
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

// The 2 N_p systems of the heatbath (Sec. IV B, eqn eofa_heatbath) for the
// poles beta[0..n_poles), LH poles first, then RH:
//   LH: H(m1) - gamma_l Delta_-(m1,m2) P_-,    RH: H(m2) - beta_l gamma_l Delta_+(m1,m2) P_+,
// gamma_l = 1/(1+beta_l), with right-hand sides Omega_-+ P_-+ eta (App. A);
// coef[r] (with alpha) the weight of the system's solution in phi:
//   phi = a_eta eta + P Omega^dag sum_r coef[r] y_r,  coef = +-alpha_l gamma_l k gamma_l.
struct HeatbathSystems {
  std::vector<eofa_system> sys;
  std::vector<double> coef, om;
  std::vector<int> chir;
  double a_eta = 0.0;
};

int heatbath_systems(eofa_ctx* C, double m1, double m2, int n_poles, const double* alpha, const double* beta,
                     HeatbathSystems& H) {
  const Geometry& g = C->g;
  const int nsys = 2 * n_poles;
  H.sys.resize(nsys);
  H.coef.assign(nsys, 0.0);
  H.om.resize((size_t)nsys * g.Ls);
  H.chir.resize(nsys);
  std::vector<double> wp(g.Ls), wm(g.Ls);
  omega_col(g.Ls, C->c, C->d, +1, wp.data());
  omega_col(g.Ls, C->c, C->d, -1, wm.data());
  const double k = k_eofa(g.Ls, C->c, C->d, m1, m2);
  H.a_eta = alpha ? alpha[0] : 0.0;
  for (int l = 0; l < n_poles; ++l) {
    const double bl = beta[l];
    if (!(1.0 + bl != 0.0) || !std::isfinite(bl)) return fail(EOFA_ERR_INVALID, "pole beta_l = -1 or non-finite");
    const double gl = 1.0 / (1.0 + bl);
    H.sys[l] = eofa_system{m1, m1, m2, -gl, -1};
    H.sys[n_poles + l] = eofa_system{m2, m1, m2, -bl * gl, +1};
    if (alpha) {
      if (!std::isfinite(alpha[l + 1])) return fail(EOFA_ERR_INVALID, "non-finite alpha_l");
      H.a_eta += alpha[l + 1] * gl;
      H.coef[l] = alpha[l + 1] * gl * k * gl;
      H.coef[n_poles + l] = -alpha[l + 1] * gl * k * gl;
    }
    H.chir[l] = -1;
    H.chir[n_poles + l] = +1;
    for (int s = 0; s < g.Ls; ++s) {
      H.om[(size_t)l * g.Ls + s] = wm[s];
      H.om[(size_t)(n_poles + l) * g.Ls + s] = wp[s];
    }
  }
  if (alpha && !std::isfinite(alpha[0])) return fail(EOFA_ERR_INVALID, "non-finite alpha_0");
  return EOFA_OK;
}

int heatbath_check(eofa_ctx* C, int32_t n_poles, const double* beta, const double* pole_tol, const void* eta,
                   const eofa_solver_params* prm, const char* who) {
  if (!C || !beta || !eta) return fail(EOFA_ERR_INVALID, std::string(who) + ": NULL argument");
  if (n_poles < 1) return fail(EOFA_ERR_INVALID, "n_poles must be >= 1");
  CHK(check_params(prm));
  if (prm->form != 0) return fail(EOFA_ERR_INVALID, std::string(who) + ": form must be 0 (Cayley)");
  if (pole_tol)
    for (int r = 0; r < 2 * n_poles; ++r)
      if (!(pole_tol[r] > 0.0)) return fail(EOFA_ERR_INVALID, "pole_tol entries must be > 0");
  return EOFA_OK;
}

// Upload the heatbath coefficients (coef, Omega columns, chiralities) into
// workspace; returns device pointers.
int heatbath_upload(eofa_ctx* C, const HeatbathSystems& H, const double** d_coef, const double** d_om,
                    const int** d_chir, hipStream_t st) {
  const int nsys = (int)H.sys.size();
  const int Ls = C->g.Ls;
  void* cdev;
  const size_t cbytes = sizeof(double) * (nsys + (size_t)nsys * Ls) + sizeof(int) * nsys;
  CHK(ws(C, "hb_coef", cbytes, &cdev));
  CHK(stage(C, cbytes));
  std::vector<unsigned char> h(cbytes);
  std::memcpy(h.data(), H.coef.data(), sizeof(double) * nsys);
  std::memcpy(h.data() + sizeof(double) * nsys, H.om.data(), sizeof(double) * nsys * Ls);
  std::memcpy(h.data() + sizeof(double) * (nsys + (size_t)nsys * Ls), H.chir.data(), sizeof(int) * nsys);
  CHK(put(C, cdev, h.data(), cbytes, st));
  *d_coef = (const double*)cdev;
  *d_om = *d_coef + nsys;
  *d_chir = (const int*)(*d_om + (size_t)nsys * Ls);
  return EOFA_OK;
}

// y_r = A_r^-1 Omega P eta for the 2 N_p heatbath systems into sol
// ([2 N_p] canonical fields): batched, or (use_guess) the poles of each side
// one after another from chronological forecasts. Returns the worst status
// of the solves (EOFA_ERR_NOT_CONVERGED passes through).
int heatbath_poles(eofa_ctx* C, const HeatbathSystems& H, const double* d_om, const int* d_chir,
                   const double* pole_tol, const void* eta, void* sol, const eofa_solver_params* prm,
                   eofa_solver_stats* sts, hipStream_t st) {
  const Geometry& g = C->g;
  const int nsys = (int)H.sys.size(), n_poles = nsys / 2;
  const size_t fbytes = (size_t)g.Ls * g.V * 12 * 16;
  void* rhs;
  CHK(ws(C, "full_rhs", fbytes * nsys, &rhs));  // shared with eofa_force
  launch_omega_rhs(g, eta, rhs, d_om, d_chir, nsys, st);
  HIPCHK(hipGetLastError());
  int rc = EOFA_OK;
  if (!prm->use_guess) {
    eofa_solver_params p2 = *prm;
    rc = solve_batch(C, H.sys.data(), nsys, rhs, sol, &p2, sts, st, pole_tol);
    if (rc != EOFA_OK && rc != EOFA_ERR_NOT_CONVERGED) return rc;
    return rc;
  }
  constexpr int max_prev = 8;
  for (int side = 0; side < 2; ++side) {
    std::vector<const void*> prev;
    for (int l = 0; l < n_poles; ++l) {
      const int r = side * n_poles + l;
      const void* rhs_r = (const char*)rhs + fbytes * r;
      void* sol_r = (char*)sol + fbytes * r;
      eofa_solver_params p2 = *prm;
      p2.use_guess = prev.empty() ? 0 : 1;
      if (!prev.empty()) CHK(forecast(C, &H.sys[r], rhs_r, prev, sol_r, st));
      const int rr = solve_batch(C, &H.sys[r], 1, rhs_r, sol_r, &p2, sts + r, st, pole_tol ? pole_tol + r : nullptr);
      if (rr != EOFA_OK && rr != EOFA_ERR_NOT_CONVERGED) return rr;
      if (rr != EOFA_OK) rc = rr;
      prev.push_back(sol_r);
      if ((int)prev.size() > max_prev) prev.erase(prev.begin());
    }
  }
  return rc;
}

}  // namespace

extern "C" int eofa_heatbath_poles(eofa_ctx* C, double m1, double m2, int32_t n_poles, const double* beta,
                                   const double* pole_tol, const void* eta, void* sol,
                                   const eofa_solver_params* prm, eofa_solver_stats* stats, void* stream) {
  CHK(heatbath_check(C, n_poles, beta, pole_tol, eta, prm, "eofa_heatbath_poles"));
  if (!sol) return fail(EOFA_ERR_INVALID, "eofa_heatbath_poles: NULL argument");
  const size_t fbytes = (size_t)C->g.Ls * C->g.V * 12 * 16;
  const char *e0 = (const char*)eta, *s0 = (const char*)sol;
  if (e0 + fbytes > s0 && s0 + fbytes * 2 * n_poles > e0)
    return fail(EOFA_ERR_INVALID, "eofa_heatbath_poles: eta and sol overlap");
  hipStream_t st = (hipStream_t)stream;
  HeatbathSystems H;
  CHK(heatbath_systems(C, m1, m2, n_poles, nullptr, beta, H));
  const double *d_coef, *d_om;
  const int* d_chir;
  CHK(heatbath_upload(C, H, &d_coef, &d_om, &d_chir, st));
  std::vector<eofa_solver_stats> st_local(2 * n_poles);
  const int rc = heatbath_poles(C, H, d_om, d_chir, pole_tol, eta, sol, prm, stats ? stats : st_local.data(), st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return rc;
}

extern "C" int eofa_heatbath_solve(eofa_ctx* C, double m1, double m2, int32_t n_poles, const double* alpha,
                                   const double* beta, const double* pole_tol, const void* eta, void* phi,
                                   const eofa_solver_params* prm, eofa_solver_stats* stats, void* stream) {
  CHK(heatbath_check(C, n_poles, beta, pole_tol, eta, prm, "eofa_heatbath_solve"));
  if (!alpha || !phi) return fail(EOFA_ERR_INVALID, "eofa_heatbath_solve: NULL argument");
  if (eta == phi) return fail(EOFA_ERR_INVALID, "eofa_heatbath_solve: eta and phi alias");
  hipStream_t st = (hipStream_t)stream;
  HeatbathSystems H;
  CHK(heatbath_systems(C, m1, m2, n_poles, alpha, beta, H));
  const double *d_coef, *d_om;
  const int* d_chir;
  CHK(heatbath_upload(C, H, &d_coef, &d_om, &d_chir, st));
  const size_t fbytes = (size_t)C->g.Ls * C->g.V * 12 * 16;
  void* sol;
  CHK(ws(C, "full_sol", fbytes * 2 * n_poles, &sol));  // shared with eofa_force
  std::vector<eofa_solver_stats> st_local(2 * n_poles);
  const int rc = heatbath_poles(C, H, d_om, d_chir, pole_tol, eta, sol, prm, stats ? stats : st_local.data(), st);
  if (rc != EOFA_OK && rc != EOFA_ERR_NOT_CONVERGED) return rc;
  launch_heatbath_combine(C->g, eta, sol, phi, H.a_eta, d_coef, d_om, d_chir, 2 * n_poles, st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return rc;
}

extern "C" int eofa_forecast(eofa_ctx* C, const eofa_system* sys, const void* rhs, const void* prev, int32_t n_prev,
                             void* guess, void* stream) {
  if (!C || !rhs || !prev || !guess) return fail(EOFA_ERR_INVALID, "eofa_forecast: NULL argument");
  if (n_prev < 1 || n_prev > 32) return fail(EOFA_ERR_INVALID, "eofa_forecast: n_prev must be 1..32");
  CHK(check_systems(sys, 1));
  const size_t fbytes = (size_t)C->g.Ls * C->g.V * 12 * 16;
  const char *g0 = (const char*)guess, *p0 = (const char*)prev, *r0 = (const char*)rhs;
  if ((g0 < p0 + fbytes * n_prev && p0 < g0 + fbytes) || (g0 < r0 + fbytes && r0 < g0 + fbytes))
    return fail(EOFA_ERR_INVALID, "eofa_forecast: guess overlaps rhs or prev");
  hipStream_t st = (hipStream_t)stream;
  std::vector<const void*> pv(n_prev);
  for (int k = 0; k < n_prev; ++k) pv[k] = p0 + fbytes * k;
  CHK(forecast(C, sys, rhs, pv, guess, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

// ---------------------------------------------------------------------------
// link derivative of the hopping term and the EOFA pseudofermion force

namespace {

DerivArgs deriv_args(eofa_ctx* C, const void* a, const void* b, void* y, double coef, int g5r5_a, int acc) {
  DerivArgs d;
  for (int k = 0; k < 4; ++k) d.L[k] = C->g.L[k];
  d.Ls = C->g.Ls;
  d.Vh = C->g.Vh;
  d.links[0] = (const double2*)C->links[P64][0];
  d.links[1] = (const double2*)C->links[P64][1];
  d.a = (const double2*)a;
  d.b = (const double2*)b;
  d.y = (double2*)y;
  d.coef = coef;
  d.g5r5_a = g5r5_a;
  d.accumulate = acc;
  return d;
}

}  // namespace

extern "C" int eofa_dhop_derivative(eofa_ctx* C, const void* a, const void* b, void* y, void* stream) {
  if (!C || !a || !b || !y) return fail(EOFA_ERR_INVALID, "eofa_dhop_derivative: NULL argument");
  if (y == a || y == b) return fail(EOFA_ERR_INVALID, "eofa_dhop_derivative: y aliases an input");
  launch_dhop_deriv(deriv_args(C, a, b, y, 1.0, 0, 0), (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return EOFA_OK;
}

extern "C" int eofa_force(eofa_ctx* C, double m1, double m2, const void* phi, void* force,
                          const eofa_solver_params* prm, eofa_solver_stats* stats, void* stream) {
  if (!C || !phi || !force) return fail(EOFA_ERR_INVALID, "eofa_force: NULL argument");
  if (phi == force) return fail(EOFA_ERR_INVALID, "eofa_force: phi and force alias");
  if (!std::isfinite(m1) || !std::isfinite(m2)) return fail(EOFA_ERR_INVALID, "eofa_force: non-finite mass");
  CHK(check_params(prm));
  if (prm->precond != 0) return fail(EOFA_ERR_INVALID, "eofa_force: precond must be 0 (batched CGNR)");
  if (prm->form != 0) return fail(EOFA_ERR_INVALID, "eofa_force: form must be 0 (Cayley)");
  hipStream_t st = (hipStream_t)stream;
  const Geometry& g = C->g;
  // chi_1 = H(m1)^-1 Omega_- P_- phi,  chi_2 = [H(m2) - Delta_+(m1,m2) P_+]^-1 Omega_+ P_+ phi
  eofa_system sys[2] = {eofa_system{m1, m1, m2, 0.0, -1}, eofa_system{m2, m1, m2, -1.0, +1}};
  std::vector<double> om(2 * g.Ls);
  omega_col(g.Ls, C->c, C->d, -1, om.data());
  omega_col(g.Ls, C->c, C->d, +1, om.data() + g.Ls);
  const int chir[2] = {-1, +1};
  const size_t fbytes = (size_t)g.Ls * g.V * 12 * 16;
  void *rhs, *chi, *cdev;
  CHK(ws(C, "full_rhs", 2 * fbytes, &rhs));  // the heatbath's buffers: canonical fields are large
  CHK(ws(C, "full_sol", 2 * fbytes, &chi));
  const size_t cbytes = sizeof(double) * 2 * g.Ls + sizeof(int) * 2;
  CHK(ws(C, "fo_coef", cbytes, &cdev));
  CHK(stage(C, cbytes));
  {
    std::vector<unsigned char> h(cbytes);
    std::memcpy(h.data(), om.data(), sizeof(double) * 2 * g.Ls);
    std::memcpy(h.data() + sizeof(double) * 2 * g.Ls, chir, sizeof(int) * 2);
    CHK(put(C, cdev, h.data(), cbytes, st));
  }
  const double* d_om = (const double*)cdev;
  const int* d_chir = (const int*)(d_om + 2 * g.Ls);
  launch_omega_rhs(g, phi, rhs, d_om, d_chir, 2, st);
  HIPCHK(hipGetLastError());
  std::vector<eofa_solver_stats> local(2);
  eofa_solver_params p2 = *prm;
  p2.use_guess = 0;  // chi_1, chi_2 live in library workspace: no guess
  const int rc = solve_batch(C, sys, 2, rhs, chi, &p2, stats ? stats : local.data(), st);
  if (rc != EOFA_OK && rc != EOFA_ERR_NOT_CONVERGED) return rc;
  // F = sum_a T^a k [ (g5 R5 chi_1)^dag dDhop chi_1 - (g5 R5 chi_2)^dag dDhop chi_2 ]
  const double k = k_eofa(g.Ls, C->c, C->d, m1, m2);
  const char* chi2 = (const char*)chi + fbytes;
  void* f2 = force;
  if (C->gparity) CHK(ws(C, "fo_f2", (size_t)4 * g.V * 9 * 16, &f2));  // doubled lattice, folded below
  launch_dhop_deriv(deriv_args(C, chi, chi, f2, k, 1, 0), st);
  launch_dhop_deriv(deriv_args(C, chi2, chi2, f2, -k, 1, 1), st);
  launch_force_project((size_t)4 * g.V, f2, st);
  if (C->gparity) launch_fold_force(C->Lx_phys, (size_t)g.L[1] * g.L[2] * g.L[3], f2, force, st);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return rc;
}

