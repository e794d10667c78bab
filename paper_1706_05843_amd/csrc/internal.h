// Internal declarations shared by the host solver and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/eofa.h"

namespace eofa {

enum Prec { P64 = 0, P32 = 1, P16 = 2 };

// Per-system fifth-dimension matrices, [NMAT][2 chiralities][Ls][Ls] doubles.
// chirality index 0 multiplies P_+ psi, index 1 multiplies P_- psi.
enum MatId {
  MAT_MEE = 0,         // M_ee = bee - cee L(m_op) + chi beta u v^T P_chi
  MAT_MEE_INV,         // M_ee^-1 (Sherman-Morrison on an LU inverse)
  MAT_MEE_T,           // M_ee^T
  MAT_MEE_INV_T,       // M_ee^-T
  MAT_MEE_INV_T_DT_T,  // M_ee^-T D~^T
  MAT_NEG_DT_T,        // -D~^T
  MAT_DT_T,            // D~^T
  MAT_DT,              // D~ = (c+d) + (c-d) L(m_op)
  MAT_DT_INV,          // D~^-1 (initial guesses: psi' = D~^-1 psi)
  MAT_DEE,             // dense form: D_ee = M_ee D~^-1 (App. B.2, same-parity block of D_EOFA + shift)
  MAT_DEE_INV,         // D_ee^-1 = D~ M_ee^-1
  MAT_DEE_T,           // D_ee^T
  MAT_DEE_INV_T,       // D_ee^-T
  NMAT
};

struct Geometry {
  int L[4];  // Lx, Ly, Lz, Lt
  int Ls;
  int V, Vh;
};

// host: build the matrices of one system; returns EOFA_OK or an error code
int build_fifth(const Geometry& g, double M5, double b5, double c5, const eofa_system& sys,
                double* out /* NMAT*2*Ls*Ls */, std::string& err);
// host: structured form of the same-parity block of one system,
//   out[0] = m_op, out[1] = chi beta k(m_a, m_b) (0 if beta = 0), out[2] = chi,
//   out[3] = 0, out[4 + s] = u_chi(m_op)_s   (App. B.2, eqn delta_rank_one)
// so that M_ee = A + out[1] u e_{s*}^T on chirality chi, A = bee - cee L(m_op),
// s* = Ls-1 (chi = +1) or 0 (chi = -1); and the Sherman-Morrison column
//   out[4 + Ls + s] = a_s = -out[1] x_s / (1 + out[1] x_{s*}),  x = A^-1 u,
// so that M_ee^-1 = (1 + a e_{s*}^T) A^-1 on chirality chi (0 if unshifted).
constexpr int SCOEF_HEAD = 4;
void build_struct(const Geometry& g, double M5, double b5, double c5, const eofa_system& sys, double* out);
// host: EOFA constant k(m_a, m_b) and the Omega_+- columns (App. A)
double k_eofa(int Ls, double c, double d, double m_a, double m_b);
void omega_col(int Ls, double c, double d, int chir, double* w /* Ls */);

// Device-side CG scalars, one entry per right-hand side (struct of arrays).
struct CgState {
  double* rr;      // |r|^2 of the normal-equation residual
  double* stop;    // stop when rr <= stop
  double* ww;      // |M p|^2
  double* alpha;
  double* beta;
  double* tol2;    // inner_tol^2 per rhs
  double* norm;    // scratch norms (FIN_NORM target)
  double* guard;   // set before FIN_INIT as a factor, made absolute there: a pass whose
                   // |r|^2 exceeds it is stopped as diverging (breakdown = 2); 0 = off
  int* iter;
  int* max_iter;
  int* halt;       // 1: this rhs does no more CG work
  int* u2run;      // 1: the x/p update of this iteration runs
  int* breakdown;  // 1: non-finite or non-positive curvature met; 2: diverging pass (guard)
};

enum FinMode { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_NORM = 3 };

// Roles of the fused hop kernel (see kernels.hip).
enum HopRole {
  ROLE_DSLASH = 0,   // out = Dhop D~ in
  ROLE_DSLASH_DAG,   // out = D~^T g5 Dhop g5 in
  ROLE_K1,           // out = D~ A (Dhop D~ in)   (A = M_ee^-1: K2 / RES then need no D~)
  ROLE_K2,           // out = B y - Dhop in, |out|^2   (in = D~ t from K1)
  ROLE_K3,           // out = A (g5 Dhop g5 in)
  ROLE_K4,           // r -= alpha (A g5Dhopg5 in + B y), |r|^2
  ROLE_K4S,          // r  = A g5Dhopg5 in + B y, |r|^2   (r in the field precision)
  ROLE_SRC,          // out = z - Dhop D~ in
  ROLE_RES,          // out = z - (B y - Dhop in), |out|^2   (in = D~ t from K1)
  ROLE_FULLRES,      // out = z - (B y + Dhop D~ in), |out|^2
  // dense (non-Cayley) form, App. B.2: off-parity blocks Dhop, same-parity D_ee dense
  ROLE_D1,           // out = A (Dhop in)
  ROLE_D2,           // out = B y - Dhop in, |out|^2
  ROLE_D3,           // out = A (g5 Dhop g5 in)
  ROLE_D4,           // r -= alpha (B y - g5Dhopg5 in), |r|^2
  ROLE_D4S,          // r  = B y - g5Dhopg5 in, |r|^2
  ROLE_DSRC,         // out = z - Dhop in
  ROLE_DRES,         // out = z - (B y - Dhop in), |out|^2
  ROLE_DFULLRES,     // out = z - (B y + Dhop in), |out|^2
  // Cayley form with the search direction held as p~ = D~ p (in = p~, already premixed)
  ROLE_K1T,          // out = D~ A (Dhop in)
  ROLE_K2T,          // out = M_ee D~^-1 y - Dhop in, |out|^2   (y = p~, in = D~ t from K1T)
  NROLE
};

struct HopArgs {
  const void* in;     // packed, parity 1-p, storage precision
  void* out;          // packed, parity p, storage precision
  const void* y;      // packed, parity p (B y term)
  const void* z;      // packed, parity p (ADDZ)
  void* r;            // packed, parity p, field precision (K4/K4S)
  const void* links;  // [Vh][8][9] complex for output parity p
  const int* nbr;     // [Vh][8] checkerboard index in parity 1-p
  const int* order;   // [Vh] traversal position -> checkerboard index (a permutation)
  const double* mats; // [nrhs][NMAT][2][Ls][Ls]
  int matA, matB;
  double cpd, cmd;    // c+d, c-d (premix)
  const double* mop;  // [nrhs] operator mass
  const double* scoef; // [nrhs][SCOEF_HEAD + 2 Ls] structured same-parity coefficients
  double bee, cee;    // (c+d)(4-M5)+1, 1-(c-d)(4-M5)
  const double* alpha;
  const int* halt;    // may be null
  double* partial;    // [nrhs][gridDim.x]
  int Vh, Ls, nrhs, rhs_block;
  int W;              // waves per work-group (1, 2 or 4)
  // optional CG step fused into a K3 (or D3) launch: work-group 0 of each RHS block
  // reduces fin_partial [nrhs][fin_nblk] (the previous launch's partial
  // sums) and applies finalize mode fin_mode to fin_S; null = none (other
  // roles ignore it)
  const double* fin_partial;
  int fin_nblk, fin_mode;
  CgState fin_S;
};

// kernel launchers (kernels.hip)
int launch_hop(int prec, int role, const HopArgs& a, hipStream_t st, int* nblk_out);
int hop_blocks(int prec, int Vh, int Ls, int W);
// default waves per work-group for Ls (at most 20 4D sites per work-group)
int default_waves(int Ls);
// LDS bytes the hop kernel of this role needs, for the precision and shape
size_t hop_lds_bytes(int prec, int role, int Ls, int W);
void launch_pack(int prec, const Geometry& g, const void* full, void* packed, int parity, int nrhs,
                 int g5r5, hipStream_t st);
void launch_unpack(int prec, const Geometry& g, const void* packed, void* full, int parity, int nrhs,
                   hipStream_t st);
void launch_gauge_pack(const Geometry& g, const void* gauge, const int bc[4], void* l64[2], void* l32[2],
                       void* l16[2], int* nbr[2], hipStream_t st);
void launch_smat(int prec, const Geometry& g, const void* in, void* out, const double* mats, int mat,
                 int nrhs, hipStream_t st);
void launch_convert(int pin, int pout, const Geometry& g, const void* in, void* out, int nrhs,
                    hipStream_t st);
void launch_axpy_to64(int pin, const Geometry& g, void* x64, const void* e, int nrhs, hipStream_t st);
void launch_zero(int prec, const Geometry& g, void* f, int nrhs, hipStream_t st);
int launch_norm2(int prec, const Geometry& g, const void* f, int nrhs, double* partial, hipStream_t st);
// ring form of the CG update: p into the next slot (alpha kept in ahist[nrhs]),
// and x += sum of kept alpha times the directions of nslots slots
// dt (optional): the direction is held as p~ = D~ p, so p~_{k+1} = D~ r + beta p~_k
// with D~ = (c+d) + (c-d) L(m_op[r]) (App. A) applied by lane exchange
struct DtArgs {
  const double* mop = nullptr;  // [nrhs] operator mass; nullptr: plain update
  double cpd = 0.0, cmd = 0.0;  // c+d, c-d
};
void launch_p_update(int ps, const Geometry& g, const void* r, const void* p, void* pn, const double* alpha,
                     const double* beta, const int* u2run, double* ahist, int nrhs, const DtArgs& dt,
                     hipStream_t st);
void launch_x_flush(int ps, const Geometry& g, void* x, const void* ring, size_t slot_bytes, int first, int nslots,
                    int R, const double* ahist, int nrhs, hipStream_t st);
// fused CG update: x in sol_prec(ps), the residual in ps (the inner precision)
void launch_cg_update(int ps, const Geometry& g, void* x, const void* r, void* p, const double* alpha,
                      const double* beta, const int* u2run, int nrhs, const DtArgs& dt, hipStream_t st);
void launch_finalize(int mode, const double* partial, int nblk, int nrhs, CgState st_, double* out,
                     hipStream_t st);

// heatbath helpers on canonical complex128 fields [nsys][Ls][V][4][3]
//   rhs[r]_s = om[r][s] P_chir[r] eta_0                      (Omega P eta, App. A)
//   phi_s    = a_eta eta_s + delta_{s,0} sum_r coef[r] P_chir[r] sum_s' om[r][s'] sol[r]_s'
void launch_omega_rhs(const Geometry& g, const void* eta, void* rhs, const double* om, const int* chir, int nsys,
                      hipStream_t st);
void launch_heatbath_combine(const Geometry& g, const void* eta, const void* sol, void* phi, double a_eta,
                             const double* coef, const double* om, const int* chir, int nsys, hipStream_t st);

size_t packed_bytes(int prec, const Geometry& g, int nrhs);
// traversal order of the hop kernels (host): position k -> checkerboard index
// i = row * Lx/2 + xh, x-rows visited in (y, z, t) blocks of up to 4^3
void site_order(const Geometry& g, int* out);
size_t link_bytes(int prec, const Geometry& g);

}  // namespace eofa

namespace eofa {
struct Buf {
  void* p = nullptr;
  size_t n = 0;
};
// bump allocation over the no-allocation scratch array for one call
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  std::map<std::string, std::pair<size_t, size_t>> slots;  // name -> (offset, bytes)
};

// records the message returned by eofa_last_error() and passes the code on
int set_error(int code, const std::string& msg);

}  // namespace eofa

// the context behind the opaque eofa_ctx handle
struct eofa_ctx {
  using Geometry = eofa::Geometry;
  using Buf = eofa::Buf;
  Geometry g;
  double M5, b5, c5, c, d;
  int bc[4];
  int device;
  void* links[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  int* nbr[2] = {nullptr, nullptr};
  int* order = nullptr;  // hop-kernel traversal order (site_order), [Vh]
  // G-parity in x: the lattice is held x-doubled (flavour f at x + f Lx) with
  // links [U, conj(U)] and an antiperiodic x edge; Lx_phys is the physical Lx
  bool gparity = false;
  int Lx_phys = 0;
  std::map<std::string, Buf> pool;
  // set only during eofa_cg_solve_noalloc: workspace and coefficients come
  // from the scratch array instead of the pool and the coefficient cache
  eofa::Arena* arena = nullptr;
  double* mats_active = nullptr;
  // fifth-dimension matrices of the last systems uploaded
  std::vector<double> sys_key;
  double* mats = nullptr;  // [nrhs][NMAT][2][Ls][Ls] then mop[nrhs]
  size_t mats_n = 0;
  double* host_stage = nullptr;  // pinned
  size_t host_stage_n = 0;
  std::vector<hipEvent_t> events;
  // autotuned (waves per work-group, right-hand sides per work-group) of the
  // inner hop kernels, keyed by precision * 4096 + nrhs
  std::map<int, std::pair<int, int>> tuned;
  hipStream_t cap_stream = nullptr;  // non-blocking stream for HIP graph capture
};

namespace eofa {
// z = N(r) for packed FP32 odd half-fields of one right-hand side (net.cpp)
int net_apply_internal(eofa_ctx* C, eofa_net* N, const void* in, void* out, hipStream_t st);
// out = M^dag M in for the odd Schur system of sys, packed FP32 odd half-fields
// of one right-hand side, FP32 arithmetic (api.cpp)
int normal_op_fp32(eofa_ctx* C, const eofa_system* sys, const void* in, void* out, hipStream_t st);
}  // namespace eofa
