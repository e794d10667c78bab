/*
 * eofa.h -- C ABI of the MI355X (gfx950) EOFA Mobius domain-wall solver.
 *
 * The library solves the generic EOFA linear system (Sec. VI A, eqn
 * generic_eofa_system, of Jung, Kelly, Mawhinney, Murphy, arXiv:1706.05843)
 *
 *     ( H(m_op) + beta * Delta_chi(m_a, m_b) P_chi ) psi = phi,
 *     H = gamma_5 R5 D_EOFA,
 *
 * for Mobius domain-wall fermions, by the paper's route: multiply by
 * gamma_5 R5 (App. B, eqn non_hermit_sys), right-precondition by D~^-1
 * (App. B.2, eqn precond_mobius_eofa_system), even-odd Schur complement on
 * the odd sublattice (App. B), CG on the normal equations, reconstruction.
 *
 * Conventions
 * -----------
 * * Lattice dims[4] = {Lx, Ly, Lz, Lt}; every entry even and >= 2; Ls even
 *   (App. A assumes even Ls), 2 <= Ls <= 32.
 * * Mobius (b5, c5): the paper's c = (b5+c5)/2, d = (b5-c5)/2; the paper
 *   fixes d = 1/2 (Sec. II), so b5 - c5 must equal 1.
 * * Gamma matrices in the chiral basis: gamma_k = [[0, -i sigma_k],
 *   [i sigma_k, 0]] (k = x, y, z), gamma_t = [[0, 1], [1, 0]],
 *   gamma_5 = diag(1, 1, -1, -1); P_+ keeps spins 0, 1.
 * * Wilson hop (Sec. II, eqn Ddwf): forward hop (1 - gamma_mu) U_mu(x),
 *   backward hop (1 + gamma_mu) U_mu(x - mu)^dag, overall -1/2; bc[mu] = +1
 *   periodic, -1 antiperiodic (applied to fermion hops across the edge).
 * * Parity of a site = (x + y + z + t) mod 2; even = 0, odd = 1.
 *
 * Canonical (user) layouts, complex128 = two doubles (re, im):
 *   gauge   [4][Lt][Lz][Ly][Lx][3][3]           row-major SU(3) links U_mu(x)
 *   fermion [nrhs][Ls][Lt][Lz][Ly][Lx][4][3]     spin then colour
 * G-parity in x (bc[0] = 2; the paper's G-parity ensembles, operator form
 * read as: two flavours, flavour 1 hopping with conj(U), fields across the x
 * edge psi(x + Lx) = [[0, 1], [-1, 0]] psi(x), links U(x + Lx) = conj(U(x))):
 *   fermion [nrhs][Ls][Lt][Lz][Ly][2][Lx][4][3]  (flavour between y and x;
 *   internally the x-doubled lattice 2Lx with links [U, conj(U)] and an
 *   antiperiodic x edge). The gauge input and the force stay physical
 *   [4][Lt][Lz][Ly][Lx][3][3]; eofa_dhop_derivative returns the doubled
 *   [4][Lt][Lz][Ly][2][Lx][3][3]. Only x may carry G-parity.
 *
 * Packed (internal) half-field of one parity: site index
 *   i = (((t*Lz + z)*Ly + y)*Lx + x) / 2,  Vh = Lx*Ly*Lz*Lt / 2,
 * components c = spin*3 + colour grouped in pairs q = c/2 (q = 0..2 is the
 * P_+ half, q = 3..5 the P_- half); element (rhs, q, s, i) at
 *   ((rhs*6 + q)*Vh + i)*Ls + s          (s fastest: one site's column is contiguous)
 * with element = two complex numbers:
 *   EOFA_FP64  : 2 x (double re, double im)      32 bytes
 *   EOFA_FP32  : 2 x (float re, float im)        16 bytes
 * EOFA_FP16S groups the components in quads j = c/4 (j = 0..2) instead:
 * element (rhs, j, s, i) at ((rhs*3 + j)*Vh + i)*Ls + s holds
 *   4 x (half re, half im)                        16 bytes, plus one float
 *   scale per 5D site at (rhs*Vh + i)*Ls + s stored after the values; the
 *   site's 24 reals are value * scale with scale = max |re|, |im| of the site.
 * eofa_packed_bytes() gives the size of one packed half-field block.
 *
 * Memory and streams
 * ------------------
 * Every field pointer is a DEVICE pointer owned by the caller (for example
 * torch tensor data_ptr()), and must not alias another argument unless
 * stated. `stream` is a hipStream_t (NULL = default stream). dslash,
 * mooee, mooee_inv, pack and unpack are asynchronous on `stream`;
 * cg_solve and heatbath_solve block until their result is on the device
 * and the stats are filled. The context owns only its internal copies of
 * the gauge field and its workspace, freed by eofa_destroy. Calls on one
 * context must not overlap (one caller thread, one stream at a time).
 *
 * Errors
 * ------
 * Every entry point returns 0 on success or a negative eofa_status; on
 * failure eofa_last_error() returns a message (thread-local, valid until
 * the next call from that thread). Nothing aborts and no exception crosses
 * the ABI.
 */
#ifndef EOFA_H
#define EOFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EOFA_OK = 0,
  EOFA_ERR_INVALID = -1,       /* bad argument: odd dims/Ls, b5-c5 != 1, |chi| != 1, null, alias */
  EOFA_ERR_NOT_CONVERGED = -2, /* solve hit max_iter / max_outer; psi holds the last iterate      */
  EOFA_ERR_BREAKDOWN = -3,     /* Sherman-Morrison denominator 0, NaN/Inf, CG breakdown            */
  EOFA_ERR_HIP = -4,           /* a HIP runtime call failed                                        */
  EOFA_ERR_OOM = -5            /* device allocation failed                                         */
} eofa_status;

typedef enum { EOFA_FP64 = 0, EOFA_FP32 = 1, EOFA_FP16S = 2 } eofa_prec;

typedef struct eofa_ctx eofa_ctx;
typedef struct eofa_net eofa_net;

/* Mobius domain-wall action (Sec. II, eqn Ddwf; Table "ensembles" for bc). */
typedef struct {
  int32_t dims[4]; /* Lx, Ly, Lz, Lt                                  */
  int32_t Ls;
  double M5, b5, c5;
  int32_t bc[4];   /* +1 periodic, -1 antiperiodic, per direction;
                      bc[0] = 2: G-parity in x (see the layouts above)    */
} eofa_action;

/* One EOFA system (eqn generic_eofa_system):
 *   (H(m_op) + beta Delta_chi(m_a, m_b) P_chi) psi = phi.
 * beta = 0 gives the plain H(m_op) system; chi is then ignored.
 * Delta_chi and k(m_a, m_b) follow App. A (Mobius kernel).            */
typedef struct {
  double m_op, m_a, m_b, beta;
  int32_t chi; /* +1 or -1 */
} eofa_system;

typedef struct {
  double tol;          /* stop when |phi - A psi| / |phi| <= tol, FP64 true residual           */
  int32_t max_iter;    /* total inner CG iterations allowed (all outer passes)                 */
  int32_t max_outer;   /* FP64 defect-correction passes (Sec. VI A); >= 1                      */
  int32_t inner_prec;  /* eofa_prec of the inner CG (FP64: plain solve)                        */
  double inner_tol;    /* floor of the inner CG stop |r_k| <= t |r_0| on the normal equations;
                          each pass uses t = max(inner_tol, 0.3 tol |phi| / |outer residual|);
                          0 = automatic floor (0 for FP64 inner, 1e-4 otherwise)               */
  int32_t fixed_iters; /* > 0: exactly this many inner iterations in one pass, no early stop   */
  int32_t check_every; /* host convergence poll period in iterations (0 = 16)                 */
  int32_t profile;     /* 1: time the inner hop kernels with HIP events (stats.hop_ms);
                          ignored when use_graph = 1                                          */
  int32_t use_graph;   /* 1: capture check_every inner iterations in a HIP graph and replay it */
  int32_t rhs_block;   /* right-hand sides per work-group in the hop kernels (links staged once
                          per work-group serve all of them); 0 = autotune                     */
  int32_t waves;       /* waves per work-group in the hop kernels (1, 2, 4); 0 = autotune
                          (rhs_block and waves both 0: the pair is timed on the first solve of
                          a shape and kept for the process, per device and lattice)          */
  int32_t precond;     /* 0: CGNR as above; 1: flexible CG on the normal equations in FP64 with
                          the learned preconditioner `net` (NULL = identity), one right-hand
                          side at a time, falling back to CGNR on breakdown or stagnation     */
  int32_t fcg_window;  /* precond = 1: previous directions each new one is A-orthogonalised
                          against (1..32; 0 = 1: the network is Hermitian positive
                          semi-definite, so one suffices; more guard against rounding)        */
  const eofa_net* net; /* precond = 1: network (eofa_net_create), evaluated in FP32             */
  int32_t use_guess;   /* 1: psi holds an initial guess on entry (canonical layout; the
                          iteration starts from psi' = D~^-1 psi on the odd sublattice)       */
  int32_t form;        /* 0: Cayley form with D~^-1 right preconditioning (App. B.2, the
                          paper's route); 1: the dense form for comparison: the EOFA matrix
                          itself, off-parity blocks Dhop and same-parity blocks the dense
                          Ls x Ls D_ee = M_ee D~^-1 per chirality (eofa_cg_solve with
                          precond = 0 only; heatbath and force reject it)                     */
  int32_t keep_direction; /* CGNR below FP64: 1 = each outer pass after the first keeps the
                          inner search direction and only replaces the residual by the FP64
                          one (a reliable update; passes then end at a residual reduction
                          of at most 0.1 for FP16S, 0.01 for FP32; a pass whose |r|^2 grows
                          1e4x is dropped and, like a pass that reduced the FP64 residual
                          less than 2x, followed by a restart); 0 = each pass restarts the
                          inner CG from p = r (plain defect correction). Pays on
                          well-conditioned systems, costs iterations on ill-conditioned ones */
  int32_t ring_slots;  /* CGNR: search directions kept for the batched solution update
                          (x += sum of alpha_j p_j every ring_slots / 2 iterations instead of
                          x += alpha p every iteration; not in the paper, memory traffic
                          only): 0 = the most of 16, 8, 4 that divide check_every (16 if 0)
                          and fit a quarter of the free device memory, else the
                          per-iteration update; 16, 8 or 4 = that many (must divide it);
                          -1 = the per-iteration update                                    */
} eofa_solver_params;

typedef struct {
  int32_t iters;        /* inner CG iterations, summed over outer passes       */
  int32_t outer_iters;  /* FP64 outer passes                                   */
  int32_t converged;    /* 1 if true_resid <= tol                              */
  int32_t status;       /* eofa_status of this right-hand side                 */
  double true_resid;    /* |b - (D_DWF + chi beta Delta~) psi'| / |b|, FP64    */
  double seconds;       /* wall time of the whole call                        */
  double hop_ms[4];     /* profile=1: summed device time of the timed inner
                           hop kernels: [0] M_ee^-1 Dhop D~, [1] M_ee - Dhop D~,
                           [2] M_ee^-T D~^T Dhop^dag, [3] residual update       */
  int32_t hop_timed;    /* profile=1: inner iterations whose kernels were timed */
  int32_t waves;        /* launch shape the inner hop kernels used: waves and   */
  int32_t rhs_block;    /* right-hand sides per work-group (autotuned or given) */
  int32_t fell_back;    /* precond = 1: 1 if the solve fell back to CGNR        */
} eofa_solver_stats;

/* Create a context: validates the action, packs the gauge field (device
 * pointer, canonical complex128 layout above) per parity with boundary
 * phases folded in. The gauge array is not retained. EOFA_ERR_INVALID if
 * Ls is odd or outside 2..32, b5 - c5 != 1, a parameter is not finite, the
 * 5D sites of one parity (Vh * Ls, x-doubled under G-parity) reach 2^28
 * (32-bit indexing and byte offsets), or the device is not a gfx950.      */
int eofa_create(const eofa_action* act, const void* gauge, void* stream, eofa_ctx** out);
int eofa_destroy(eofa_ctx* ctx);
const char* eofa_last_error(void);

/* Bytes of one packed half-field block for nrhs right-hand sides.        */
size_t eofa_packed_bytes(const eofa_ctx* ctx, int32_t prec, int32_t nrhs);

/* Canonical full field -> packed half-field of one parity (and back).
 * g5r5 = 1 applies gamma_5 R5 on the way (App. B: b = gamma_5 R5 phi). */
int eofa_pack(eofa_ctx* ctx, const void* full, void* packed, int32_t parity, int32_t prec,
              int32_t nrhs, int32_t g5r5, void* stream);
int eofa_unpack(eofa_ctx* ctx, const void* packed, void* full, int32_t parity, int32_t prec,
                int32_t nrhs, void* stream);

/* Off-parity block of D_DWF(m_op) (eqn Ddwf minus its site-local part):
 *   out_p = Dhop_{p <- 1-p} D~(m_op) in_{1-p},   D~ = (c+d) + (c-d) L(m_op)
 * (dagger = 1: out_p = D~^T gamma_5 Dhop gamma_5 in, its adjoint). in and
 * out are packed half-fields of parities 1-out_parity and out_parity;
 * sys[r] gives m_op for right-hand side r.                               */
int eofa_dslash(eofa_ctx* ctx, const eofa_system* sys, const void* in, void* out,
                int32_t out_parity, int32_t dagger, int32_t prec, int32_t nrhs, void* stream);

/* Same-parity block of the Cayley-form operator (App. B.2):
 *   M_ee = ((c+d)(4-M5)+1) - (1-(c-d)(4-M5)) L(m_op) + chi beta u_chi v_chi^T P_chi
 * (eqn delta_rank_one), site local; out = M_ee in (dagger: M_ee^T in).   */
int eofa_mooee(eofa_ctx* ctx, const eofa_system* sys, const void* in, void* out, int32_t dagger,
               int32_t prec, int32_t nrhs, void* stream);

/* out = M_ee^-1 in (dagger: M_ee^-T in); the inverse is built per system
 * with Sherman-Morrison (eqn sherman_morrison_mobius_inv). Fails with
 * EOFA_ERR_BREAKDOWN if the Sherman-Morrison denominator vanishes.       */
int eofa_mooee_inv(eofa_ctx* ctx, const eofa_system* sys, const void* in, void* out,
                   int32_t dagger, int32_t prec, int32_t nrhs, void* stream);

/* Solve nrhs independent EOFA systems sys[r] for canonical phi[r] -> psi[r]
 * (device, complex128, canonical layout; psi is output only unless
 * params->use_guess = 1, then it is also the initial guess). Inner CG in
 * params->inner_prec with an FP64 defect-correction outer loop (Sec. VI A);
 * every inner CG vector (search direction, residual, operator
 * intermediates) is stored in the inner precision, the inner solution
 * increment in FP32 (FP64 for an FP64 inner solve); all right-hand sides
 * iterate together in batched kernels, each with its own CG scalars.
 * stats: host array [nrhs] (may be NULL).                                */
int eofa_cg_solve(eofa_ctx* ctx, const eofa_system* sys, const void* phi, void* psi, int32_t nrhs,
                  const eofa_solver_params* params, eofa_solver_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code around which they
 * capture HIP graphs of their own work, tight serving loops, harnesses that
 * forbid hipMalloc): eofa_cg_solve with precond = 0 (and use_graph = 0) whose
 * workspace (packed fields, partial sums, CG scalars, the systems'
 * coefficients) comes from a fixed 64 MiB device array held by the library
 * on each GPU until the process ends, instead of from allocations. It calls
 * no hipMalloc / hipFree / hipHostMalloc and creates no stream or event:
 * host staging was set aside by eofa_create. Same kernels and results as
 * eofa_cg_solve with the same params; waves = rhs_block = 0 take the default
 * launch shape (no autotuning), profile is ignored, the direction ring is
 * used only if it fits beside the other buffers. Returns EOFA_ERR_INVALID
 * (before any device work) when the lattice and nrhs need more than the
 * 64 MiB. Every call on a GPU uses that GPU's one array and leaves its
 * contents behind (each call writes every buffer before reading it): calls
 * that overlap on one GPU (other threads, other streams, other contexts)
 * race and must not be issued. The context's device must be current.      */
int eofa_cg_solve_noalloc(eofa_ctx* ctx, const eofa_system* sys, const void* phi, void* psi, int32_t nrhs,
                          const eofa_solver_params* params, eofa_solver_stats* stats, void* stream);

/* EOFA heatbath (Sec. IV B, eqn eofa_heatbath): phi = f(M_EOFA) eta for
 * the rational f(x) = alpha[0] + sum_l alpha[l] / (beta[l-1] + x),
 * l = 1..n_poles, via the 2*n_poles systems
 *   LH: (H(m1) - gamma_l Delta_-(m1,m2) P_-),  RH: (H(m2) - beta_l gamma_l Delta_+(m1,m2) P_+),
 * gamma_l = 1/(1+beta_l). eta, phi: device canonical complex128 fields (one
 * right-hand side). alpha: host [n_poles+1], beta: host [n_poles].
 * pole_tol: host [2*n_poles] FP64 true-residual target per system (LH poles
 * then RH; Sec. VI B per-pole tuning), or NULL for params->tol everywhere.
 * params->use_guess = 0: all systems in one batched solve; 1: the poles of
 * each side one after another, each started from the chronological forecast
 * (Sec. VI B, after Brower et al.) over up to 8 previous solutions of that
 * side. stats: host [2*n_poles] (LH poles then RH), may be NULL.         */
int eofa_heatbath_solve(eofa_ctx* ctx, double m1, double m2, int32_t n_poles, const double* alpha,
                        const double* beta, const double* pole_tol, const void* eta, void* phi,
                        const eofa_solver_params* params, eofa_solver_stats* stats, void* stream);

/* The 2*n_poles pole solutions of the heatbath (Sec. IV B, eqn
 * eofa_heatbath) before they are combined into phi:
 *   sol[l]           = [H(m1) - gamma_l Delta_-(m1,m2) P_-]^-1 Omega_- P_- eta,
 *   sol[n_poles + l] = [H(m2) - beta_l gamma_l Delta_+(m1,m2) P_+]^-1 Omega_+ P_+ eta,
 * gamma_l = 1/(1+beta_l), l = 0..n_poles-1 (Omega_+- as in App. A; the
 * right-hand sides take eta at s = 0 only). sol: device, 2*n_poles
 * canonical fields in the layout of eta, one after another; it must not
 * overlap eta. beta, pole_tol, params and stats as for
 * eofa_heatbath_solve (the same route: batched, or poles in sequence from
 * chronological forecasts). EOFA_ERR_NOT_CONVERGED if a system misses its
 * target (its solution is still written). Blocks until done.            */
int eofa_heatbath_poles(eofa_ctx* ctx, double m1, double m2, int32_t n_poles, const double* beta,
                        const double* pole_tol, const void* eta, void* sol,
                        const eofa_solver_params* params, eofa_solver_stats* stats, void* stream);

/* Chronological forecast (Sec. VI B, after Brower et al.): the initial
 * guess sum_k c_k prev_k for the system sys with right-hand side rhs, over
 * n_prev (1..32) earlier solutions, from the Galerkin conditions
 *   sum_k c_k prev_l^dag A prev_k = prev_l^dag rhs   for every l,
 * A = H(m_op) + beta Delta_chi(m_a,m_b) P_chi (eqn generic_eofa_system): the
 * minimiser of psi^dag A psi - rhs^dag psi - psi^dag rhs on their span.
 * rhs, guess: device canonical fields; prev: n_prev canonical fields one
 * after another; guess must not overlap rhs or prev. The n_prev x n_prev
 * system is solved on the host; if it is numerically singular the guess is
 * zero. Blocks until done.                                               */
int eofa_forecast(eofa_ctx* ctx, const eofa_system* sys, const void* rhs, const void* prev, int32_t n_prev,
                  void* guess, void* stream);

/* Link derivative of the hopping term (Sec. IV C): for canonical 5D fields
 * a, b (device complex128, one right-hand side) and every link (x, mu), the
 * 3 x 3 complex matrix y_mu(x) such that
 *   a^dag (d/ds Dhop(U_mu(x) -> e^{s T} U_mu(x)))|_{s=0} b = Tr(T y_mu(x))
 * for every traceless anti-Hermitian T (Dhop with its -1/2 and the boundary
 * phases, eqn Ddwf). y: device complex128 [4][Lt][Lz][Ly][Lx][3][3], the
 * gauge layout; it must not alias a or b. Asynchronous on `stream`.       */
int eofa_dhop_derivative(eofa_ctx* ctx, const void* a, const void* b, void* y, void* stream);

/* EOFA pseudofermion force (Sec. IV C, eqn eofa_force): for every link
 *   F_mu(x) = sum_a T^a d/ds S(U_mu(x) -> e^{s T^a} U_mu(x))|_{s=0},
 *   S = phi^dag M_EOFA phi (eqn eofa_action), T^a = i lambda^a / 2,
 * i.e. F^a = k (g5 R5 chi_1)^dag dDhop chi_1 - k (g5 R5 chi_2)^dag dDhop chi_2
 * with chi_1 = H(m1)^-1 Omega_- P_- phi and
 * chi_2 = [H(m2) - Delta_+(m1,m2) P_+]^-1 Omega_+ P_+ phi, both solved in one
 * batched call with `params` (precond must be 0). phi: device canonical
 * complex128 field (only its s = 0 slice enters, through Omega). force:
 * device complex128 gauge layout, traceless anti-Hermitian matrices.
 * stats: host [2] (chi_1, chi_2) or NULL. Blocks until done.              */
int eofa_force(eofa_ctx* ctx, double m1, double m2, const void* phi, void* force,
               const eofa_solver_params* params, eofa_solver_stats* stats, void* stream);

/* Training pairs for the learned preconditioner (not in the paper). Runs
 * FP64 CG on the normal equations A x = M^dag b~ (A = M^dag M, odd Schur
 * system of sys, one right-hand side phi in the canonical layout) from
 * x = 0, records at iterations k = first, first+stride, ... the residual
 * r_k = M^dag b~ - A x_k and the error e_k = x* - x_k, where x* is the same
 * CG continued to |r| <= tol |r_0| (x_k is kept in FP64 until x* is known).
 * r_out, e_out: device, npairs consecutive packed FP32 odd half-fields
 * (eofa_packed_bytes(ctx, EOFA_FP32, 1) bytes each). *recorded (host) is
 * the number of pairs written (fewer than npairs if CG converges first);
 * *iters (host, may be NULL) the CG iterations to x*.
 * EOFA_ERR_NOT_CONVERGED if max_iter iterations do not reach tol.        */
int eofa_cg_pairs(eofa_ctx* ctx, const eofa_system* sys, const void* phi, int32_t npairs, int32_t first,
                  int32_t stride, double tol, int32_t max_iter, void* r_out, void* e_out, int32_t* recorded,
                  int32_t* iters, void* stream);

/* Learned preconditioner (not in the paper): N = B^dag B with B a stack of
 * n_layers gauge-covariant parallel-transport layers, channels
 * channels[0..n_layers] (channels[0] = channels[n_layers] = 1, each 1..8).
 * Layer l maps C_in to C_out channels on the full lattice with 20 terms
 * per channel pair, each a complex weight times a gauge-covariant operator:
 *   y_c = sum_c' sum_t W[t][c][c'] S_t X_c',
 *   S_0 = P_+, S_1 = P_-   (same site; P_+- = (1 +- g5)/2)
 *   S_{2+mu} = T_{+mu}, S_{6+mu} = T_{-mu},
 *   S_{10+mu} = g_mu T_{+mu}, S_{14+mu} = g_mu T_{-mu},
 *   (S_18 X)(x, s) = P_+ X(x, s-1), (S_19 X)(x, s) = P_- X(x, s+1) (cyclic in s),
 *   T_{+mu} X(x) = U_mu(x) X(x+mu), T_{-mu} X(x) = U_mu(x-mu)^dag X(x-mu)
 * (fermion boundary phases on edge hops; g_mu in the chiral basis of the
 * field layout). B^dag applies the adjoint layers in reverse order, so N
 * is Hermitian and positive semi-definite (<x, N x> = |B x|^2). The input
 * is an odd packed FP32 half-field embedded with zero even sites; the
 * output is the odd half of B^dag B of it. Weights: FP32 master copy (Adam
 * state beside it), used as bfloat16 in the kernels, FP32 arithmetic;
 * stored layer by layer as W[20][C_out][C_in] complex (re, im).
 * A network holds device memory only; it may be used with any context
 * whose lattice matches the one it was last applied on (buffers are
 * resized otherwise). Initial weights: N(0, s^2) real and imaginary parts,
 * s = init_scale / sqrt(20 C_in), from `seed`, plus 1 on W[0][0][0] and
 * W[1][0][0] (the identity from channel 0 to channel 0), so that an
 * untrained network is close to the identity.                           */
int eofa_net_create(eofa_ctx* ctx, int32_t n_layers, const int32_t* channels, uint64_t seed,
                    double init_scale, eofa_net** out);
int eofa_net_destroy(eofa_net* net);
/* complex weights in total; get/set exchange 2 * that many doubles (host) */
size_t eofa_net_num_weights(const eofa_net* net);
int eofa_net_get_weights(const eofa_net* net, double* out);
int eofa_net_set_weights(eofa_net* net, const double* in); /* also resets Adam */
/* out = N(in): packed FP32 odd half-fields (one right-hand side), no alias */
int eofa_net_apply(eofa_ctx* ctx, eofa_net* net, const void* in, void* out, void* stream);
/* Loss over npairs consecutive packed FP32 odd half-fields (device) and its
 * gradient dL/dW* (Wirtinger; the gradient in (Re W, Im W) is twice its real
 * and imaginary parts) as host grad[2 * num_weights] (may be NULL); loss:
 * host (may be NULL). Two losses:
 *   sys == NULL: error loss     sum_p |N(r_p) - e_p|^2 / |e_p|^2  (pairs r, e);
 *   sys != NULL: residual loss  sum_p min_c |c A N(r_p) - r_p|^2 / |r_p|^2
 *                = sum_p [1 - |<A y_p, r_p>|^2 / (|A y_p|^2 |r_p|^2)],
 *                y_p = N(r_p), A = M^dag M of the odd Schur system of sys
 *                (applied by the hop kernels in FP32): the best scale c is
 *                taken out because CG does not depend on the scale of its
 *                preconditioner; e is not used and may be NULL. A pair with
 *                A y_p = 0 contributes 1 and no gradient.                */
int eofa_net_loss_grad(eofa_ctx* ctx, eofa_net* net, const eofa_system* sys, const void* r, const void* e,
                       int32_t npairs, double* loss, double* grad, void* stream);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * pairs, in order, in mini-batches of `batch`; one step per mini-batch on
 * the batch-mean loss (sys selects the loss as above). loss_per_epoch: host
 * [epochs] mean loss per pair over the epoch, measured during it (may be
 * NULL).                                                                 */
int eofa_net_train(eofa_ctx* ctx, eofa_net* net, const eofa_system* sys, const void* r, const void* e,
                   int32_t npairs, int32_t epochs, int32_t batch, double lr, double* loss_per_epoch,
                   void* stream);

/* Host only (no device work): the fifth-dimension matrix `mat` that the
 * library builds for one system, as out[2][Ls][Ls] (row-major; [0] acts on
 * P_+ psi, [1] on P_- psi). mat: 0 M_ee, 1 M_ee^-1, 2 M_ee^T, 3 M_ee^-T,
 * 4 M_ee^-T D~^T, 5 -D~^T, 6 D~^T, 7 D~, 8 D~^-1, and the dense form's
 * 9 D_ee = M_ee D~^-1, 10 D_ee^-1, 11 D_ee^T, 12 D_ee^-T (App. A, App. B.2).
 * Returns EOFA_ERR_BREAKDOWN if the Sherman-Morrison denominator vanishes. */
int eofa_fifth_matrix(const eofa_action* act, const eofa_system* sys, int32_t mat, double* out);

#ifdef __cplusplus
}
#endif
#endif
