// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts).
//
// Operators (Sec. II, eqn Ddwf; App. B):
//   Dhop psi(x) = -1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//   D~ = (c+d) + (c-d) L(m):  (D~ psi)_s = (c+d) psi_s + (c-d) (P_+ (L_+ psi)_s + P_- (L_- psi)_s)
//   (L_+ psi)_s = psi_{s-1} (s >= 1), -m psi_{Ls-1} (s = 0);  (L_- psi)_s = psi_{s+1}, -m psi_0 at Ls-1
// The off-parity block of D_DWF is Dhop D~; its adjoint is D~^T g5 Dhop g5, and
// g5 Dhop g5 is Dhop with (1 -+ g_mu) swapped.
//
// Layout: see include/eofa.h. One thread owns one 5D site (i, s); a work-group
// holds SB consecutive 4D sites with their whole Ls column, so
//  * the 8 links of each 4D site are staged once in LDS and reused by all Ls
//    threads of that site and by every right-hand side of the block;
//  * the Ls x Ls fifth-dimension epilogues (M_ee^-1, M_ee, D~^T) exchange the
//    column through LDS.
// Spin projection: in the chiral basis g_mu = [[0, A_mu], [A_mu^dag, 0]], so
// (1 + sg g_mu) psi = [h ; sg A^dag h] with h = psi_up + sg A psi_lo: the link
// multiplies a 2-spinor only.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "device_common.h"
#include "internal.h"

namespace eofa {

// ---------------------------------------------------------------------------
// the fused hop kernel

// epilogue applied to the hop result h = Dhop (D~ in) of each 5D site:
//   A_ID    v = h              A_NEG  v = -h
//   A_MAT   v = M h            (dense Ls x Ls per chirality, through LDS)
//   A_DTT   v = D~^T h         A_NDTT v = -D~^T h   (structured: lane exchange)
//   A_MATDT v = M D~^T h
//   A_DMINV v = D~ M_ee^-1 h   A_MINVDT v = M_ee^-T D~^T h   (the inverse
//           structured along the column: minv_rows for Ls = 16, minv_cols
//           otherwise; D~ and D~^T by lane exchange)
// plus the same-site term B y:
//   B_MEE   + M_ee y           B_MEET + M_ee^T y    (structured: lane exchange)
//   B_MEE_DTI + M_ee D~^-1 y   (y = p~ = D~ p; D~^-1 a geometric series along s)
enum { A_ID = 0, A_NEG = 1, A_MAT = 2, A_DTT = 3, A_NDTT = 4, A_MATDT = 5, A_DMINV = 6, A_MINVDT = 7 };
enum { B_NONE = 0, B_MEE = 1, B_MEET = 2, B_DENSE = 3, B_MEE_DTI = 4 };
enum { O_STORE = 0, O_ADDZ = 1, O_RUPD = 2, O_STORE_R = 3 };

template <int ROLE>
struct RoleT;
#define EOFA_ROLE(NAME, dag, pre, am, bm, om, nrm)   \
  template <>                                        \
  struct RoleT<NAME> {                               \
    static constexpr bool DAG = dag, PRE = pre;      \
    static constexpr int AM = am;                    \
    static constexpr int BM = bm;                    \
    static constexpr int OM = om;                    \
    static constexpr bool NRM = nrm;                 \
  };
EOFA_ROLE(ROLE_DSLASH, false, true, A_ID, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_DSLASH_DAG, true, false, A_DTT, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_K1, false, true, A_DMINV, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_K2, false, false, A_NEG, B_MEE, O_STORE, true)
EOFA_ROLE(ROLE_K3, true, false, A_MINVDT, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_K4, true, false, A_NDTT, B_MEET, O_RUPD, true)
EOFA_ROLE(ROLE_K4S, true, false, A_NDTT, B_MEET, O_STORE_R, true)
EOFA_ROLE(ROLE_SRC, false, true, A_ID, B_NONE, O_ADDZ, false)
EOFA_ROLE(ROLE_RES, false, false, A_NEG, B_MEE, O_ADDZ, true)
EOFA_ROLE(ROLE_FULLRES, false, true, A_ID, B_MEE, O_ADDZ, true)
// dense (non-Cayley) form: off-parity blocks Dhop alone, same-parity blocks dense
EOFA_ROLE(ROLE_D1, false, false, A_MAT, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_D2, false, false, A_NEG, B_DENSE, O_STORE, true)
EOFA_ROLE(ROLE_D3, true, false, A_MAT, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_D4, true, false, A_NEG, B_DENSE, O_RUPD, true)
EOFA_ROLE(ROLE_D4S, true, false, A_NEG, B_DENSE, O_STORE_R, true)
EOFA_ROLE(ROLE_DSRC, false, false, A_ID, B_NONE, O_ADDZ, false)
EOFA_ROLE(ROLE_DRES, false, false, A_NEG, B_DENSE, O_ADDZ, true)
EOFA_ROLE(ROLE_DFULLRES, false, false, A_ID, B_DENSE, O_ADDZ, true)
// the search direction held as p~ = D~ p: no premix in K1, D~^-1 on the same-site term of K2
EOFA_ROLE(ROLE_K1T, false, false, A_DMINV, B_NONE, O_STORE, false)
EOFA_ROLE(ROLE_K2T, false, false, A_NEG, B_MEE_DTI, O_STORE, true)
#undef EOFA_ROLE

constexpr int LSTR = 73;  // padded link stride per site in LDS (complex units)
constexpr int NSTR = 9;   // padded neighbour stride per site in LDS
constexpr int MAXW = 4;   // most waves per work-group

// A wave holds the whole s-columns of G = 64 / Ls consecutive 4D sites
// (lane = g * Ls + s); a work-group holds W(Ls) waves, at most 20 4D sites,
// which bounds the LDS staging of links and columns.
__host__ __device__ inline int sites_per_wave(int Ls) { return 64 / Ls; }

int default_waves(int Ls) {
  const int G = sites_per_wave(Ls);
  return G <= 5 ? MAXW : (16 / G > 1 ? 16 / G : 1);
}

template <class R>
struct HopLds {
  // byte sizes of the LDS regions
  static __host__ __device__ size_t links(int SBk) { return (size_t)SBk * LSTR * sizeof(cx<R>); }
  static __host__ __device__ size_t nbr(int SBk) { return (((size_t)SBk * NSTR * 4 + 15) / 16) * 16; }
  static __host__ __device__ size_t mat(int Ls) { return (((size_t)2 * Ls * (Ls + 1) * sizeof(R) + 15) / 16) * 16; }
  static __host__ __device__ size_t col(int SBk, int Ls) { return (size_t)SBk * (Ls * 6 + 1) * sizeof(cx<R>); }
};

// One direction's neighbour spinor as loaded: FP16S keeps the raw half2
// words and the site scale (decoded inside the arithmetic), else the values.
template <int P>
struct DirIn {
  cx<typename ST<P>::R> v[12];
};
template <>
struct DirIn<P16> {
  unsigned w[12];
  float sc;
};

// Rotation across the 16 lanes of a DPP row: lane l of each row receives the
// value of lane (l - K) mod 16 of the same row. With Ls = 16 a row is exactly
// one site's s-column (lane = g * 16 + s), so the fifth-dimension neighbour
// s - K (cyclic) costs one VALU move instead of an LDS permute.
template <int K>
__device__ __forceinline__ int row_ror(int v) {
  if constexpr ((K & 15) == 0) {
    return v;
  } else {
    // a rotation has no out-of-range source lane, so bound_ctrl (0 for such
    // lanes) changes nothing; with it set the compiler folds the move into the
    // VALU instruction that consumes it (one v_fmac_f32_dpp instead of two)
    return __builtin_amdgcn_update_dpp(0, v, 0x120 + (K & 15), 0xF, 0xF, true);
  }
}
template <int K>
__device__ __forceinline__ unsigned row_ror(unsigned v) { return (unsigned)row_ror<K>((int)v); }
template <int K>
__device__ __forceinline__ float row_ror(float v) { return __int_as_float(row_ror<K>(__float_as_int(v))); }
template <int K>
__device__ __forceinline__ double row_ror(double v) {
  const int2 w = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(row_ror<K>(w.x), row_ror<K>(w.y)));
}
template <int K, class R>
__device__ __forceinline__ cx<R> row_ror(cx<R> v) { return {row_ror<K>(v.r), row_ror<K>(v.i)}; }

// value of lane s - 1 (UP) or s + 1 (!UP) of this site's column: a DPP
// rotation when the column is a 16-lane row (RL = 16), else a lane permute
template <int RL, bool UP, class T>
__device__ __forceinline__ T col_nbr(T v, int src) {
  if constexpr (RL == 16) {
    return row_ror<UP ? 1 : 15>(v);
  } else {
    return __shfl(v, src, 64);
  }
}

template <int P>
__device__ __forceinline__ void load_dir(const void* in, const FD& fin, int r, int s, int n, DirIn<P>& b) {
  if constexpr (P == P16) {
    b.sc = scale_ptr(in, fin)[sidx(fin, r, s, n)];
    ld_words16(in, fin, r, s, n, b.w);
  } else {
    ld_spinor<P>(in, fin, r, s, n, b.v);
  }
}

// FP16S gathers through buffer descriptors: one per quad plane of the
// field and right-hand side, and one for its scales, so a gathered site
// costs one 32-bit offset per lane (shared by its three quads and, shifted,
// its scale) instead of four 64-bit address additions. The offsets are below
// 16 x Vh x Ls bytes, which the host keeps under 4 GiB (kMaxSites16).
constexpr int kBufDword3 = 0x00020000;  // raw buffer, 32-bit data format
struct Buf16 {
  __amdgpu_buffer_rsrc_t v[3], sc;
};
__device__ __forceinline__ Buf16 buf16(const void* base, const FD& f, int r) {
  const size_t qs = qstride(f);
  Buf16 B;
#pragma unroll
  for (int j = 0; j < 3; ++j)
    B.v[j] = __builtin_amdgcn_make_buffer_rsrc((char*)base + ((size_t)r * 3 + j) * qs * 16, (short)0, -1,
                                               kBufDword3);
  B.sc = __builtin_amdgcn_make_buffer_rsrc((char*)scale_ptr(base, f) + (size_t)r * qs * 4, (short)0, -1,
                                           kBufDword3);
  return B;
}
// the FP16S spinor of column site n, fifth-dimension index s
__device__ __forceinline__ void load_dir16(const Buf16& B, int Ls, int s, int n, DirIn<P16>& b) {
  const unsigned e = (unsigned)(n * Ls + s);
  b.sc = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(B.sc, e * 4u, 0, 0));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const u4v_t q = __builtin_amdgcn_raw_buffer_load_b128(B.v[j], e * 16u, 0, 0);
    b.w[4 * j] = q.x;
    b.w[4 * j + 1] = q.y;
    b.w[4 * j + 2] = q.z;
    b.w[4 * j + 3] = q.w;
  }
}

// FP16S: neighbour spinors and links stay in half precision through the
// SU(3) products. Each link element sits in LDS as the two half2 words
// (Re u, -Im u) and (Im u, Re u), so that one complex multiply-accumulate
// of u and a projected half-spinor component h = (Re h, Im h) is two
// v_dot2_f32_f16 (FP16 products, exact in FP32, summed in FP32):
//   Re += (Re u, -Im u) . h,   Im += (Im u, Re u) . h.
// The projection (1 +- g_mu) and the D~ premix run on packed halves; the
// premix is taken in units of the largest of the three site scales involved
// (own, s-1, s+1), so every factor is at most 1 and no half overflows. The
// unit multiplies the FP32 products as they are accumulated.
// YPRE: the last direction has nothing left to prefetch, so its free buffer
// takes the same-site spinor of a.y that the epilogue needs (yout).
// FP16S gather: directions whose loads are in flight ahead of the one being
// computed, and the occupancy (waves per SIMD) the register budget is set for
constexpr int kPfd16 = 1;
constexpr int kOcc16 = 5;

// SU(3) products on the matrix cores (MF): v_mfma_f32_4x4x4_16b_f16 runs 16
// independent 4x4x4 products per wave, block b on lanes 4b .. 4b+3, lane 4b+j
// supplying column j of B (its own 4 halves) and row j of A, and receiving
// column j of D (D register q = row q). When the 4 lanes of every block hold
// 5D sites of one 4D site (Ls a multiple of 4), they share each link, so
// A = the real form of U (rows (Re, Im) of each output colour, columns
// (Re, Im) of each input colour: the 2x2 blocks (Re u, -Im u; Im u, Re u)
// staged in LDS) and B = the lane's own projected half spinor give each lane
// its own U h. Per half spinor: top rows (Re, Im of colours 0, 1) and bottom
// rows (colour 2, its two rows repeated on lanes 2, 3 of the block), each
// over the K blocks (colours 0, 1) and (colour 2, zero): four products, in
// place of 18 v_dot2 on the vector ALU. Same FP16 products, FP32 sums.
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned u2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h4_t h4_of(unsigned lo, unsigned hi) { return __builtin_bit_cast(h4_t, u2_t{lo, hi}); }
__device__ __forceinline__ h4_t h4_of(h2_t lo, h2_t hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3); }

// g = U h for the two projected half spinors h[0..2], h[3..5] of one
// direction on the matrix cores. Uw: the direction's 9 staged entries (entry
// e: word 2e = (Re u, -Im u), word 2e + 1 = (Im u, Re u)); top, bot: this
// lane's word offsets of its A rows (lane j of its block: row j of the top
// blocks = colour j / 2, Re or Im by j % 2; of the bottom blocks = colour 2,
// Re or Im by j % 2). The K columns that meet B's zero halves take another
// (finite) link word.
__device__ __forceinline__ void su3_mfma(const unsigned* Uw, int top, int bot, const h2_t* h, cx<float>* gv) {
  const unsigned* Ut = Uw + top;
  const unsigned* Ub = Uw + bot;
  const h4_t A00 = h4_of(Ut[0], Ut[2]), A01 = h4_of(Ut[4], Ut[2]);
  const h4_t A10 = h4_of(Ub[12], Ub[14]), A11 = h4_of(Ub[16], Ub[14]);
  const h2_t z2 = {(_Float16)0.f, (_Float16)0.f};
  const f4_t z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const h4_t B0 = h4_of(h[k * 3], h[k * 3 + 1]), B1 = h4_of(h[k * 3 + 2], z2);
    f4_t t = __builtin_amdgcn_mfma_f32_4x4x4f16(A00, B0, z4, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_4x4x4f16(A01, B1, t, 0, 0, 0);
    f4_t b = __builtin_amdgcn_mfma_f32_4x4x4f16(A10, B0, z4, 0, 0, 0);
    b = __builtin_amdgcn_mfma_f32_4x4x4f16(A11, B1, b, 0, 0, 0);
    gv[k * 3] = {t[0], t[1]};
    gv[k * 3 + 1] = {t[2], t[3]};
    gv[k * 3 + 2] = {b[0], b[1]};
  }
}

// the same products as v_dot2 on the vector ALU (any Ls); U: the direction's
// 9 staged entries as word pairs
__device__ __forceinline__ void su3_dot2(const uint2* U, const h2_t* h, cx<float>* gv) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int a3 = 0; a3 < 3; ++a3) {
      // first product in the three-operand form with an inline zero
      // accumulator (the two-operand form would need a register cleared first)
      const uint2 u0 = U[a3 * 3];
      const unsigned h0 = __builtin_bit_cast(unsigned, h[k * 3]);
      float re, im;
      asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(re) : "v"(u0.x), "v"(h0));
      asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(im) : "v"(u0.y), "v"(h0));
#pragma unroll
      for (int b3 = 1; b3 < 3; ++b3) {
        const uint2 u = U[a3 * 3 + b3];
        re = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, u.x), h[k * 3 + b3], re, false);
        im = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2_t, u.y), h[k * 3 + b3], im, false);
      }
      gv[k * 3 + a3] = {re, im};
    }
#pragma unroll
  for (int c = 0; c < 6; ++c) asm volatile("" : "+v"(gv[c].r), "+v"(gv[c].i));
}

template <bool DAG, bool PRE, int RL, bool YPRE, bool MF>
__device__ __forceinline__ void hop_site_h(const HopArgs& a, const FD& fin, int r, int s, int g, int ls,
                                           const cx<float>* s_link, const int* s_nbr, cx<float>* acc,
                                           DirIn<P16>& yout, float fold) {
  const int Ls = a.Ls;
  float aup = 0.f, alo = 0.f, post = -0.5f;
  int src_up = 0, src_lo = 0;
  if constexpr (PRE) {
    const float q = (float)(a.cmd / a.cpd);
    const float m = (float)a.mop[r];
    post = (float)(-0.5 * a.cpd);
    aup = s > 0 ? q : -m * q;
    alo = s < Ls - 1 ? q : -m * q;
    src_up = g * Ls + (s > 0 ? s - 1 : Ls - 1);
    src_lo = g * Ls + (s < Ls - 1 ? s + 1 : 0);
  }
  post *= fold;
  // word offsets of this lane's A rows in a direction's 9 staged entries
  // (for the matrix-core products)
  const int mj = threadIdx.x & 3;
  const int mf_top = 6 * (mj >> 1) + (mj & 1), mf_bot = mj & 1;
  (void)mf_top;
  (void)mf_bot;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
  // the neighbour spinors of the next kPfd16 directions are in flight while
  // one direction is computed (kPfd16 + 1 buffers in registers)
  DirIn<P16> buf[kPfd16 + 1];
  const Buf16 bin = buf16(a.in, fin, r);
#pragma unroll
  for (int d = 0; d < kPfd16; ++d) load_dir16(bin, Ls, s, s_nbr[ls * NSTR + d], buf[d]);
#pragma unroll
  for (int dir = 0; dir < 8; ++dir) {
    __builtin_amdgcn_sched_barrier(0);
    if (dir + kPfd16 < 8)
      load_dir16(bin, Ls, s, s_nbr[ls * NSTR + dir + kPfd16], buf[(dir + kPfd16) % (kPfd16 + 1)]);
    if constexpr (YPRE) {
      if (dir + kPfd16 == 8) load_dir16(buf16(a.y, fin, r), Ls, s, s_nbr[ls * NSTR + 8], yout);
    }
    // the next directions' loads leave before this direction's data is
    // touched: without this fence the scheduler hoists the lane exchanges of
    // this direction (which wait for its loads) above them, and nothing overlaps
    __builtin_amdgcn_sched_barrier(0);
    const DirIn<P16>& b = buf[dir % (kPfd16 + 1)];
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    const float sc = b.sc;
    h2_t x[12];
    float unit;
    if constexpr (PRE) {
      // (D~ psi)_s / (c+d) = sc h_s + aup su h_{s-1} (upper) / + alo sl h_{s+1} (lower)
      const float su = col_nbr<RL, true>(sc, src_up) * aup, sl = col_nbr<RL, false>(sc, src_lo) * alo;
      unit = fmaxf(sc, fmaxf(fabsf(su), fabsf(sl)));
      unit = unit > 0.f ? unit : 1.f;
      const float inv = __builtin_amdgcn_rcpf(unit);
      const _Float16 f0 = (_Float16)(sc * inv), fu = (_Float16)(su * inv), fl = (_Float16)(sl * inv);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const unsigned t = c < 6 ? col_nbr<RL, true>(b.w[c], src_up) : col_nbr<RL, false>(b.w[c], src_lo);
        const h2_t hs = __builtin_bit_cast(h2_t, b.w[c]), ht = __builtin_bit_cast(h2_t, t);
        x[c] = (c < 6 ? fu : fl) * ht + f0 * hs;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) x[c] = __builtin_bit_cast(h2_t, b.w[c]);
      unit = sc;  // sc = 0: the halves are all zero, and so is the product
    }
    // (1 + sg g_mu) projection on packed halves (sg = -1 for (1 - g_mu));
    // i v = (-Im v, Re v)
    const bool neg = fwd != DAG;
    h2_t h[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const h2_t u0 = x[c], u1 = x[3 + c], l0 = x[6 + c], l1 = x[9 + c];
      const h2_t il0 = {-l0.y, l0.x}, il1 = {-l1.y, l1.x};
      if (mu == 0) {  // u0 - sg i l1, u1 - sg i l0
        h[c] = neg ? u0 + il1 : u0 - il1;
        h[3 + c] = neg ? u1 + il0 : u1 - il0;
      } else if (mu == 1) {  // u0 - sg l1, u1 + sg l0
        h[c] = neg ? u0 + l1 : u0 - l1;
        h[3 + c] = neg ? u1 - l0 : u1 + l0;
      } else if (mu == 2) {  // u0 - sg i l0, u1 + sg i l1
        h[c] = neg ? u0 + il0 : u0 - il0;
        h[3 + c] = neg ? u1 - il1 : u1 + il1;
      } else {  // u0 + sg l0, u1 + sg l1
        h[c] = neg ? u0 - l0 : u0 + l0;
        h[3 + c] = neg ? u1 - l1 : u1 + l1;
      }
    }
    cx<float> gv[6];
    if constexpr (MF)
      su3_mfma((const unsigned*)(s_link + ls * LSTR + dir * 9), mf_top, mf_bot, h, gv);
    else
      su3_dot2((const uint2*)(s_link + ls * LSTR + dir * 9), h, gv);
    // acc += post unit [g ; sg A^dag g] (the overall -1/2, or -(c+d)/2, and
    // the epilogue's leading factor folded into each direction's unit)
    const float ps = unit * post, ms = neg ? -ps : ps;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<float> g0 = gv[c], g1 = gv[3 + c];
      acc[c] = cfma_r(ps, g0, acc[c]);
      acc[3 + c] = cfma_r(ps, g1, acc[3 + c]);
      if (mu == 0) {  // A^dag g = (i g1, i g0)
        acc[6 + c] = cfma_r(ms, mul_i(g1), acc[6 + c]);
        acc[9 + c] = cfma_r(ms, mul_i(g0), acc[9 + c]);
      } else if (mu == 1) {  // A^dag g = (g1, -g0)
        acc[6 + c] = cfma_r(ms, g1, acc[6 + c]);
        acc[9 + c] = cfma_r(-ms, g0, acc[9 + c]);
      } else if (mu == 2) {  // A^dag g = (i g0, -i g1)
        acc[6 + c] = cfma_r(ms, mul_i(g0), acc[6 + c]);
        acc[9 + c] = cfma_r(-ms, mul_i(g1), acc[9 + c]);
      } else {
        acc[6 + c] = cfma_r(ms, g0, acc[6 + c]);
        acc[9 + c] = cfma_r(ms, g1, acc[9 + c]);
      }
    }
  }
}

// Dhop (or g5 Dhop g5 when DAG) applied to D~ in (PRE) at the 5D site (s, i)
// of local site ls. The D~ premix needs P_+ psi at s-1 and P_- psi at s+1 of
// the same neighbour: the lanes (g, s-1) and (g, s+1) of this wave hold
// exactly those spinors for the same direction, so they are exchanged across
// lanes instead of being loaded again.
template <int P, bool DAG, bool PRE, int RL, bool YPRE>
__device__ __forceinline__ void hop_site(const HopArgs& a, const FD& fin, int r, int s, int g, int ls,
                                         const cx<typename ST<P>::R>* s_link, const int* s_nbr,
                                         cx<typename ST<P>::R>* acc, DirIn<P16>& yout,
                                         typename ST<P>::R fold) {
  if constexpr (P == P16) {
    // the matrix-core products need each 4-lane block inside one column
    hop_site_h<DAG, PRE, RL, YPRE, RL == 16 || RL == 4>(a, fin, r, s, g, ls, s_link, s_nbr, acc, yout, fold);
    return;
  } else {
  using R = typename ST<P>::R;
  const int Ls = a.Ls;
  // D~ psi = (c+d) [psi_s + (c-d)/(c+d) (P_+ (L_+ psi)_s + P_- (L_- psi)_s)]: the
  // overall (c+d) is folded into the final -1/2.
  R aup = R(0), alo = R(0), post = R(-0.5);
  int src_up = 0, src_lo = 0;
  if constexpr (PRE) {
    const R q = (R)(a.cmd / a.cpd);
    const R m = (R)a.mop[r];
    post = (R)(-0.5 * a.cpd);
    aup = s > 0 ? q : -m * q;
    alo = s < Ls - 1 ? q : -m * q;
    src_up = g * Ls + (s > 0 ? s - 1 : Ls - 1);
    src_lo = g * Ls + (s < Ls - 1 ? s + 1 : 0);
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
  // Below FP64 the next direction's loads are issued before this
  // direction's arithmetic (two directions in registers), so each wave keeps
  // memory requests in flight while it computes; FP64 keeps one direction
  // live (its register budget) and relies on occupancy.
  constexpr bool PF = P != P64;
  DirIn<P> b0, b1;
  if constexpr (PF) load_dir<P>(a.in, fin, r, s, s_nbr[ls * NSTR], b0);
#pragma unroll
  for (int dir = 0; dir < 8; ++dir) {
    // scheduling fence per direction: bounds the live registers
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (PF) {
      if (dir < 7) load_dir<P>(a.in, fin, r, s, s_nbr[ls * NSTR + dir + 1], (dir & 1) ? b0 : b1);
      __builtin_amdgcn_sched_barrier(0);  // the loads leave first (as in the FP16S path)
    }
    const DirIn<P>& b = (PF && (dir & 1)) ? b1 : b0;
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    cx<R> sp[12];
    if constexpr (PF) {
#pragma unroll
      for (int c = 0; c < 12; ++c) sp[c] = b.v[c];
    } else {
      ld_spinor<P>(a.in, fin, r, s, s_nbr[ls * NSTR + dir], sp);
    }
    if constexpr (PRE) {
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const R f = c < 6 ? aup : alo;
        const cx<R> t = c < 6 ? cx<R>{col_nbr<RL, true>(sp[c].r, src_up), col_nbr<RL, true>(sp[c].i, src_up)}
                              : cx<R>{col_nbr<RL, false>(sp[c].r, src_lo), col_nbr<RL, false>(sp[c].i, src_lo)};
        sp[c] = {fma(f, t.r, sp[c].r), fma(f, t.i, sp[c].i)};
      }
    }
    // sg = -1 for (1 - g_mu), +1 for (1 + g_mu)
    const R sg = (fwd != DAG) ? R(-1) : R(1);
    cx<R> h[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> u0 = sp[c], u1 = sp[3 + c], l0 = sp[6 + c], l1 = sp[9 + c];
      if (mu == 0) {  // A = -i sigma_1
        h[c] = u0 - sg * mul_i(l1);
        h[3 + c] = u1 - sg * mul_i(l0);
      } else if (mu == 1) {  // A = -i sigma_2
        h[c] = u0 - sg * l1;
        h[3 + c] = u1 + sg * l0;
      } else if (mu == 2) {  // A = -i sigma_3
        h[c] = u0 - sg * mul_i(l0);
        h[3 + c] = u1 + sg * mul_i(l1);
      } else {  // A = 1
        h[c] = u0 + sg * l0;
        h[3 + c] = u1 + sg * l1;
      }
    }
    const cx<R>* U = s_link + ls * LSTR + dir * 9;
    cx<R> gv[6];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3) {
        cx<R> v = cmul(U[a3 * 3 + 0], h[k * 3 + 0]);
        v = cfma(U[a3 * 3 + 1], h[k * 3 + 1], v);
        v = cfma(U[a3 * 3 + 2], h[k * 3 + 2], v);
        gv[k * 3 + a3] = v;
      }
#pragma unroll
    for (int c = 0; c < 6; ++c) asm volatile("" : "+v"(gv[c].r), "+v"(gv[c].i));
    // acc += [g ; sg A^dag g]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> g0 = gv[c], g1 = gv[3 + c];
      acc[c] = acc[c] + g0;
      acc[3 + c] = acc[3 + c] + g1;
      if (mu == 0) {  // A^dag g = (i g1, i g0)
        acc[6 + c] = acc[6 + c] + sg * mul_i(g1);
        acc[9 + c] = acc[9 + c] + sg * mul_i(g0);
      } else if (mu == 1) {  // A^dag g = (g1, -g0)
        acc[6 + c] = acc[6 + c] + sg * g1;
        acc[9 + c] = acc[9 + c] - sg * g0;
      } else if (mu == 2) {  // A^dag g = (i g0, -i g1)
        acc[6 + c] = acc[6 + c] + sg * mul_i(g0);
        acc[9 + c] = acc[9 + c] - sg * mul_i(g1);
      } else {
        acc[6 + c] = acc[6 + c] + sg * g0;
        acc[9 + c] = acc[9 + c] + sg * g1;
      }
    }
  }
  post *= fold;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = post * acc[c];
  }
}

template <class R>
__device__ __forceinline__ void load_mat(R* dst, const double* src, int Ls, int tid, int nthr) {
  // src: [2][Ls][Ls] doubles -> dst rows padded to Ls+1
  for (int j = tid; j < 2 * Ls * Ls; j += nthr) {
    const int ch = j / (Ls * Ls), rem = j % (Ls * Ls), row = rem / Ls, col = rem % Ls;
    dst[(ch * Ls + row) * (Ls + 1) + col] = (R)src[j];
  }
}

// out(s) for one chirality half: v[c] = sum_s' M[ch][s][s'] col[s'][c]
template <class R>
__device__ __forceinline__ void col_matvec(const R* M, const cx<R>* col, int Ls, int s, int half,
                                           cx<R>* v, bool accumulate) {
  const R* row = M + (half * Ls + s) * (Ls + 1);
  cx<R> t[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) t[c] = accumulate ? v[half * 6 + c] : cx<R>{R(0), R(0)};
  for (int sp = 0; sp < Ls; ++sp) {
    const R m = row[sp];
    const cx<R>* src = col + sp * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      t[c].r = fma(m, src[c].r, t[c].r);
      t[c].i = fma(m, src[c].i, t[c].i);
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) v[half * 6 + c] = t[c];
}

template <class R>
__device__ __forceinline__ cx<R> shfl_cx(cx<R> v, int src) {
  return {__shfl(v.r, src, 64), __shfl(v.i, src, 64)};
}

// Fifth-dimension neighbours of lane (g, s) in its wave: the column of one 4D
// site lives in lanes g*Ls .. g*Ls+Ls-1.
//   (L_+ v)_s = v_{s-1}, -m v_{Ls-1} at s = 0;  (L_- v)_s = v_{s+1}, -m v_0 at s = Ls-1
//   L_+^T has the L_- pattern and L_-^T the L_+ pattern.
template <class R>
struct SNbr {
  int sp, sn;  // source lanes of s-1 and s+1 (cyclic)
  R fp, fn;    // 1, or -m across the wrap
};

template <class R, bool TRANS, int RL>
__device__ __forceinline__ void lmul(const cx<R>* v, cx<R>* out, const SNbr<R>& nb) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const cx<R> t = TRANS ? cx<R>{col_nbr<RL, false>(v[c].r, nb.sn), col_nbr<RL, false>(v[c].i, nb.sn)}
                          : cx<R>{col_nbr<RL, true>(v[c].r, nb.sp), col_nbr<RL, true>(v[c].i, nb.sp)};
    out[c] = (TRANS ? nb.fn : nb.fp) * t;
  }
#pragma unroll
  for (int c = 6; c < 12; ++c) {
    const cx<R> t = TRANS ? cx<R>{col_nbr<RL, true>(v[c].r, nb.sp), col_nbr<RL, true>(v[c].i, nb.sp)}
                          : cx<R>{col_nbr<RL, false>(v[c].r, nb.sn), col_nbr<RL, false>(v[c].i, nb.sn)};
    out[c] = (TRANS ? nb.fp : nb.fn) * t;
  }
}

// z += k (L y) (TRANS: k (L^T y)) in the generic column form: the wrap factor
// rides on the coefficient, one FMA per real component. z may alias y: each
// component's neighbour value is read before that component is written.
template <class R, bool TRANS, int RL>
__device__ __forceinline__ void lacc(cx<R>* z, const cx<R>* y, const SNbr<R>& nb, R k) {
  const R kp = nb.fp * k, kn = nb.fn * k;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const cx<R> t = TRANS ? cx<R>{col_nbr<RL, false>(y[c].r, nb.sn), col_nbr<RL, false>(y[c].i, nb.sn)}
                          : cx<R>{col_nbr<RL, true>(y[c].r, nb.sp), col_nbr<RL, true>(y[c].i, nb.sp)};
    const R f = TRANS ? kn : kp;
    z[c] = {fma(f, t.r, z[c].r), fma(f, t.i, z[c].i)};
  }
#pragma unroll
  for (int c = 6; c < 12; ++c) {
    const cx<R> t = TRANS ? cx<R>{col_nbr<RL, true>(y[c].r, nb.sp), col_nbr<RL, true>(y[c].i, nb.sp)}
                          : cx<R>{col_nbr<RL, false>(y[c].r, nb.sn), col_nbr<RL, false>(y[c].i, nb.sn)};
    const R f = TRANS ? kp : kn;
    z[c] = {fma(f, t.r, z[c].r), fma(f, t.i, z[c].i)};
  }
}

// v[half] (+)= M v'[half] for the Ls x Ls matrix of chirality `half` (rows
// padded to Ls + 1 in LDS), Ls = 16: the sum over s' runs along the cyclic
// diagonals, M[s][s-k] times the value of lane s-k brought by a row rotation,
// so the column never goes through LDS
template <class R, int K>
__device__ __forceinline__ void diag_step(const R* M, const cx<R>* src, int s, int half, cx<R>* t) {
  // one diagonal at a time: unfenced, the scheduler hoists all 16 rotations
  // and their LDS reads together and the live values spill
  __builtin_amdgcn_sched_barrier(0);
  const R d = M[(half * 16 + s) * 17 + ((s - K) & 15)];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const cx<R> v = row_ror<K>(src[half * 6 + c]);
    t[c].r = fma(d, v.r, t[c].r);
    t[c].i = fma(d, v.i, t[c].i);
  }
}
template <class R, int K = 0>
__device__ __forceinline__ void diag_steps(const R* M, const cx<R>* src, int s, int half, cx<R>* t) {
  if constexpr (K < 16) {
    diag_step<R, K>(M, src, s, half, t);
    diag_steps<R, K + 1>(M, src, s, half, t);
  }
}
template <class R>
__device__ __forceinline__ void row_matvec(const R* M, const cx<R>* src, int s, cx<R>* v, bool accumulate) {
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    cx<R> t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c] = accumulate ? v[half * 6 + c] : cx<R>{R(0), R(0)};
    diag_steps<R>(M, src, s, half, t);
    // the sums are complete here: the rotations are convergent and cannot
    // follow the arithmetic into the (live-lane) store branch, so without
    // this fence every rotated value stays live across it and spills
#pragma unroll
    for (int c = 0; c < 6; ++c) asm volatile("" : "+v"(t[c].r), "+v"(t[c].i));
#pragma unroll
    for (int c = 0; c < 6; ++c) v[half * 6 + c] = t[c];
  }
}

// sum over the 16 lanes of each row, left in every lane
template <class R>
__device__ __forceinline__ cx<R> row_sum(cx<R> v) {
  v = v + row_ror<8>(v);
  v = v + row_ror<4>(v);
  v = v + row_ror<2>(v);
  return v + row_ror<1>(v);
}

// z <- (1 + rho^N L^N) z on the 6 components of one chirality half, Ls = 16.
// UP: L = L_+ ((L z)_s = z_{s-1}, -m z_{15} at s = 0), a rotation by N;
// else L = L_- ((L z)_s = z_{s+1}, -m z_0 at s = 15), a rotation by 16 - N.
// Lanes whose source wraps around the column take the factor -m.
// z[c] += f * (z[c] of lane (l - K) mod 16 of the same row) for the six complex
// values of one chirality half, as twelve v_fmac_f32_dpp: the rotation rides
// on the multiply-accumulate (the compiler folds a rotation into a multiply or
// an add but not into v_fmac). The result is the same FMA as fma(f, t, z). A
// DPP read of a VGPR needs two wait states after a VALU write of it, and the
// compiler does not see the reads and writes inside the statement: s_nop 1 on
// both sides covers the instruction before it and the one after it; inside,
// every source was last written by the previous statement.
#define EOFA_FMAC_ROR_1(K, n) "v_fmac_f32_dpp %" #n ", %" #n ", %12 row_ror:" #K " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define EOFA_FMAC_ROR(K)                                                                                    \
  asm("s_nop 1\n\t" EOFA_FMAC_ROR_1(K, 0) EOFA_FMAC_ROR_1(K, 1) EOFA_FMAC_ROR_1(K, 2) EOFA_FMAC_ROR_1(K, 3) \
      EOFA_FMAC_ROR_1(K, 4) EOFA_FMAC_ROR_1(K, 5) EOFA_FMAC_ROR_1(K, 6) EOFA_FMAC_ROR_1(K, 7)                 \
      EOFA_FMAC_ROR_1(K, 8) EOFA_FMAC_ROR_1(K, 9) EOFA_FMAC_ROR_1(K, 10) EOFA_FMAC_ROR_1(K, 11) "s_nop 1"      \
      : "+v"(z[0].r), "+v"(z[0].i), "+v"(z[1].r), "+v"(z[1].i), "+v"(z[2].r), "+v"(z[2].i), "+v"(z[3].r),     \
        "+v"(z[3].i), "+v"(z[4].r), "+v"(z[4].i), "+v"(z[5].r), "+v"(z[5].i)                                  \
      : "v"(f))
template <int K>
__device__ __forceinline__ void fmac_ror6(cx<float>* z, float f) {
  static_assert(K == 1 || K == 2 || K == 4 || K == 8 || K == 12 || K == 14 || K == 15, "rotation");
  if constexpr (K == 1) EOFA_FMAC_ROR(1);
  else if constexpr (K == 2) EOFA_FMAC_ROR(2);
  else if constexpr (K == 4) EOFA_FMAC_ROR(4);
  else if constexpr (K == 8) EOFA_FMAC_ROR(8);
  else if constexpr (K == 12) EOFA_FMAC_ROR(12);
  else if constexpr (K == 14) EOFA_FMAC_ROR(14);
  else EOFA_FMAC_ROR(15);
}
#undef EOFA_FMAC_ROR
#undef EOFA_FMAC_ROR_1

// z[c] += f * (y[c] of lane (l - K) mod 16 of the same row), y another array:
// twelve v_fmac_f32_dpp with the rotated y as the DPP source (wait states as
// above: y may have been written just before, z is read by DPP just after)
#define EOFA_FMACS_1(K, n, m) "v_fmac_f32_dpp %" #n ", %" #m ", %24 row_ror:" #K " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
#define EOFA_FMACS(K)                                                                                          \
  asm("s_nop 1\n\t" EOFA_FMACS_1(K, 0, 12) EOFA_FMACS_1(K, 1, 13) EOFA_FMACS_1(K, 2, 14) EOFA_FMACS_1(K, 3, 15) \
      EOFA_FMACS_1(K, 4, 16) EOFA_FMACS_1(K, 5, 17) EOFA_FMACS_1(K, 6, 18) EOFA_FMACS_1(K, 7, 19)                 \
      EOFA_FMACS_1(K, 8, 20) EOFA_FMACS_1(K, 9, 21) EOFA_FMACS_1(K, 10, 22) EOFA_FMACS_1(K, 11, 23) "s_nop 1"     \
      : "+v"(z[0].r), "+v"(z[0].i), "+v"(z[1].r), "+v"(z[1].i), "+v"(z[2].r), "+v"(z[2].i), "+v"(z[3].r),         \
        "+v"(z[3].i), "+v"(z[4].r), "+v"(z[4].i), "+v"(z[5].r), "+v"(z[5].i)                                      \
      : "v"(y[0].r), "v"(y[0].i), "v"(y[1].r), "v"(y[1].i), "v"(y[2].r), "v"(y[2].i), "v"(y[3].r), "v"(y[3].i),    \
        "v"(y[4].r), "v"(y[4].i), "v"(y[5].r), "v"(y[5].i), "v"(f))
template <int K>
__device__ __forceinline__ void fmac_ror6_from(cx<float>* z, const cx<float>* y, float f) {
  static_assert(K == 1 || K == 15, "rotation");
  if constexpr (K == 1) EOFA_FMACS(1);
  else EOFA_FMACS(15);
}
#undef EOFA_FMACS
#undef EOFA_FMACS_1

// z += k (L y) on one chirality half, Ls = 16 rows: UP L = L_+ ((L y)_s =
// y_{s-1}, -m y_15 at s = 0), else L = L_- (y_{s+1}, -m y_0 at s = 15)
template <bool UP>
__device__ __forceinline__ void lacc_rows(cx<float>* z, const cx<float>* y, int s, float k, float m) {
  const bool wrap = UP ? s == 0 : s == 15;
  fmac_ror6_from<UP ? 1 : 15>(z, y, wrap ? -m * k : k);
}

template <class R, int N, bool UP>
__device__ __forceinline__ void scan_step(cx<R>* z, int s, R rhoN, R m) {
  const bool wrap = UP ? s < N : s > 15 - N;
  const R f = wrap ? -m * rhoN : rhoN;
  if constexpr (sizeof(R) == 4) {
    fmac_ror6<UP ? N : 16 - N>(z, f);
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cx<R> t = row_ror<UP ? N : 16 - N>(z[c]);
      z[c].r = fma(f, t.r, z[c].r);
      z[c].i = fma(f, t.i, z[c].i);
    }
  }
}

// z <- sum_{k<16} (x L)^k z on a 16-lane row (Ls = 16; L^16 = -m), by four
// doublings (1 + x^8 L^8)(1 + x^4 L^4)(1 + x^2 L^2)(1 + x L); x1 = x, x2 = x^2, ...
template <class R, bool UP>
__device__ __forceinline__ void series_rows(cx<R>* z, int s, R x1, R x2, R x4, R x8, R m) {
  scan_step<R, 1, UP>(z, s, x1, m);
  scan_step<R, 2, UP>(z, s, x2, m);
  scan_step<R, 4, UP>(z, s, x4, m);
  scan_step<R, 8, UP>(z, s, x8, m);
}

// Structured inverse of the same-parity block on a 16-lane row (App. B.2):
// A = bee (1 - rho L), rho = cee / bee, and L^16 = -m, so
//   A^-1 = (1 + rho^8 L^8)(1 + rho^4 L^4)(1 + rho^2 L^2)(1 + rho L) / (bee (1 + m rho^16))
// (the geometric series of rho L, summed in four doublings); the EOFA shift
// adds the rank-one Sherman-Morrison term on the shifted chirality:
//   M_ee^-1 = (1 + a e_{s*}^T) A^-1,   M_ee^-T = A^-T (1 + e_{s*} a^T),
// with a_s from the host. A^-T uses L^T, which for L_+ is L_- in structure
// and vice versa. TRANS selects M_ee^-T. About 250 VALU operations per lane
// instead of the 768 of the dense Ls x Ls product.
// 1/x: the hardware reciprocal (1 ulp) in FP32, a division in FP64
template <class R>
__device__ __forceinline__ R recip(R x) {
  if constexpr (sizeof(R) == 4)
    return __builtin_amdgcn_rcpf(x);
  else
    return R(1) / x;
}

template <class R, bool TRANS, bool NORM = true>
__device__ __forceinline__ void minv_rows(cx<R>* v, int s, int g, R bee, R cee, R m, R sk, int chi, R a_s) {
  const R rho = cee * recip(bee);
  const R rho2 = rho * rho, rho4 = rho2 * rho2, rho8 = rho4 * rho4, rho16 = rho8 * rho8;
  const R scale = NORM ? recip(bee * (R(1) + m * rho16)) : R(1);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    cx<R>* z = v + half * 6;
    const int chir = half == 0 ? 1 : -1;
    const bool shifted = sk != R(0) && chi == chir;  // uniform over the block
    const int star = g * 16 + (chir > 0 ? 15 : 0);
    if constexpr (TRANS) {
      if (shifted) {  // z_{s*} += sum_s a_s z_s
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const cx<R> t = row_sum(a_s * z[c]);
          if (s == (chir > 0 ? 15 : 0)) z[c] = z[c] + t;
        }
      }
    }
    // A^-1 uses L_chi; A^-T the other direction
    if ((chir > 0) != TRANS)
      series_rows<R, true>(z, s, rho, rho2, rho4, rho8, m);
    else
      series_rows<R, false>(z, s, rho, rho2, rho4, rho8, m);
    if constexpr (NORM) {
#pragma unroll
      for (int c = 0; c < 6; ++c) z[c] = scale * z[c];
    }
    if constexpr (!TRANS) {
      if (shifted) {  // z += a z_{s*}
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const cx<R> zs = {__shfl(z[c].r, star, 64), __shfl(z[c].i, star, 64)};
          z[c].r = fma(a_s, zs.r, z[c].r);
          z[c].i = fma(a_s, zs.i, z[c].i);
        }
      }
    }
  }
}

// z <- sum_{k<Ls} (x L)^k z for any Ls by lane permutes within the column
// (lanes g*Ls .. g*Ls+Ls-1; L^Ls = -m; up: L = L_+, lane s takes s - j, else
// L_-, s + j), as a product over the prime factors p_i of Ls:
//   sum_{k<Ls} y^k = prod_i (1 + y^{n_i} + ... + y^{(p_i - 1) n_i}),  n_i = p_1 ... p_{i-1}
template <class R>
__device__ __forceinline__ void series_cols(cx<R>* z, int s, int g, int Ls, R x, R m, bool up) {
  int n = 1, rest = Ls;
  R rn = x;  // x^n
  while (rest > 1) {
    int p = 2;
    while (rest % p != 0) ++p;
    cx<R> add[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) add[c] = {R(0), R(0)};
    R rj = R(1);
    for (int k = 1; k < p; ++k) {
      const int j = k * n;
      rj *= rn;
      const int t = up ? s - j : s + j;
      const bool wrap = up ? t < 0 : t >= Ls;
      const int src = g * Ls + (wrap ? (up ? t + Ls : t - Ls) : t);
      const R f = wrap ? -m * rj : rj;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const cx<R> w = {__shfl(z[c].r, src, 64), __shfl(z[c].i, src, 64)};
        add[c].r = fma(f, w.r, add[c].r);
        add[c].i = fma(f, w.i, add[c].i);
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) z[c] = z[c] + add[c];
    rn *= rj;  // x^(n p) = x^n x^((p - 1) n)
    n *= p;
    rest /= p;
  }
}

// v <- D~^-1 v (App. A): per chirality D~ = (c+d)(1 + q L) with q = (c-d)/(c+d)
// (L_+ on P_+ psi, L_- on P_- psi) and L^Ls = -m, so for even Ls
//   D~^-1 = sum_{k<Ls} (-q L)^k / ((c+d)(1 + m q^Ls)).
template <class R, int RL, bool NORM = true>
__device__ __forceinline__ void dtinv(cx<R>* v, int s, int g, int Ls, R cpd, R cmd, R m) {
  const R q = cmd * recip(cpd), x1 = -q;
  R qLs = R(1);
  for (int k = 0; k < Ls; ++k) qLs *= q;
  const R scale = NORM ? recip(cpd * (R(1) + m * qLs)) : R(1);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    cx<R>* z = v + half * 6;
    if constexpr (RL == 16) {
      const R x2 = x1 * x1, x4 = x2 * x2, x8 = x4 * x4;
      if (half == 0)
        series_rows<R, true>(z, s, x1, x2, x4, x8, m);
      else
        series_rows<R, false>(z, s, x1, x2, x4, x8, m);
    } else {
      series_cols<R>(z, s, g, Ls, x1, m, half == 0);
    }
    if constexpr (NORM) {
#pragma unroll
      for (int c = 0; c < 6; ++c) z[c] = scale * z[c];
    }
  }
}

// the normalisations the structured inverses leave to their callers:
// 1/(bee (1 + m rho^Ls)), rho = cee/bee, of M_ee^-1 (unshifted part), and
// 1/((c+d)(1 + m q^Ls)), q = (c-d)/(c+d), of D~^-1
template <class R>
__device__ __forceinline__ R power_ls(R x, int Ls) {  // x^Ls by squaring
  R p = R(1), b = x;
  for (int e = Ls; e > 0; e >>= 1) {
    if (e & 1) p *= b;
    b *= b;
  }
  return p;
}
template <class R>
__device__ __forceinline__ R minv_norm(R bee, R cee, R m, int Ls) {
  return recip(bee * (R(1) + m * power_ls(cee * recip(bee), Ls)));
}
template <class R>
__device__ __forceinline__ R dtinv_norm(R cpd, R cmd, R m, int Ls) {
  return recip(cpd * (R(1) + m * power_ls(cmd * recip(cpd), Ls)));
}

// The same structured inverse for any Ls, by lane permutes within the
// column (lanes g*Ls .. g*Ls+Ls-1). The geometric series of x = rho L is
// summed as a product over the prime factors p_1 p_2 ... of Ls:
//   sum_{k<Ls} x^k = prod_i (1 + x^{n_i} + ... + x^{(p_i - 1) n_i}),
//   n_i = p_1 ... p_{i-1},
// one pass of p_i - 1 shifted copies per factor (every shift below Ls; L^j
// takes lane s - j, or s + j in the other direction, times -m across the
// wrap). Ls = 12 = 2 2 3 takes 4 shifted copies per component instead of
// the 12-term dense product. The rank-one term as in minv_rows; the
// transposed form's sum over s' goes through the column's LDS slot.
template <class R, bool TRANS, bool NORM = true>
__device__ __forceinline__ void minv_cols(cx<R>* v, int s, int g, int Ls, R bee, R cee, R m, R sk, int chi, R a_s,
                                          cx<R>* mycol, bool in_col) {
  const R rho = cee * recip(bee);
  R rhoLs = R(1);
  for (int k = 0; k < Ls; ++k) rhoLs *= rho;
  const R scale = NORM ? recip(bee * (R(1) + m * rhoLs)) : R(1);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    cx<R>* z = v + half * 6;
    const int chir = half == 0 ? 1 : -1;
    const bool shifted = sk != R(0) && chi == chir;  // uniform over the block
    const int star_s = chir > 0 ? Ls - 1 : 0;
    if constexpr (TRANS) {
      if (shifted) {  // z_{s*} += sum_s a_s z_s
        __syncthreads();
        if (in_col)
#pragma unroll
          for (int c = 0; c < 6; ++c) mycol[s * 6 + c] = a_s * z[c];
        __syncthreads();
        if (in_col && s == star_s) {
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            cx<R> t = {R(0), R(0)};
            for (int q = 0; q < Ls; ++q) t = t + mycol[q * 6 + c];
            z[c] = z[c] + t;
          }
        }
      }
    }
    // A^-1 uses L_chi (lane s takes s - j for L_+, s + j for L_-); A^-T the other
    series_cols<R>(z, s, g, Ls, rho, m, (chir > 0) != TRANS);
    if constexpr (NORM) {
#pragma unroll
      for (int c = 0; c < 6; ++c) z[c] = scale * z[c];
    }
    if constexpr (!TRANS) {
      if (shifted) {  // z += a z_{s*}
        const int star = g * Ls + star_s;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const cx<R> zs = {__shfl(z[c].r, star, 64), __shfl(z[c].i, star, 64)};
          z[c].r = fma(a_s, zs.r, z[c].r);
          z[c].i = fma(a_s, zs.i, z[c].i);
        }
      }
    }
  }
}

// Rank-one part of the shifted same-parity block on the chirality half H0
// (0: P_+, 6: P_-), with s* the special fifth-dimension index:
//   TRANS = false:  v_s += sk u_s y_{s*}              (sk u e_{s*}^T y)
//   TRANS = true :  v_s += delta_{s,s*} sk sum_s' u_s' y_s'   (sk e_{s*} u^T y)
template <class R, bool TRANS, int H0, int RL>
__device__ __forceinline__ void rank_one(const cx<R>* y, cx<R>* v, R sk, R us, int star_lane, bool is_star,
                                         cx<R>* mycol, int s, int Ls, bool in_col) {
  if constexpr (TRANS && RL == 16) {  // the sum over s' along the row, no LDS
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cx<R> sum = row_sum(us * y[H0 + c]);
      if (is_star) {
        v[H0 + c].r = fma(sk, sum.r, v[H0 + c].r);
        v[H0 + c].i = fma(sk, sum.i, v[H0 + c].i);
      }
    }
  } else if constexpr (!TRANS) {
    const R f = sk * us;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cx<R> ys = shfl_cx(y[H0 + c], star_lane);
      v[H0 + c].r = fma(f, ys.r, v[H0 + c].r);
      v[H0 + c].i = fma(f, ys.i, v[H0 + c].i);
    }
  } else {
    __syncthreads();
    if (in_col)
#pragma unroll
      for (int c = 0; c < 6; ++c) mycol[s * 6 + c] = us * y[H0 + c];
    __syncthreads();
    if (in_col && is_star) {  // idle lanes past the last column read no slot
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        cx<R> sum = {R(0), R(0)};
        for (int q = 0; q < Ls; ++q) sum = sum + mycol[q * 6 + c];
        v[H0 + c].r = fma(sk, sum.r, v[H0 + c].r);
        v[H0 + c].i = fma(sk, sum.i, v[H0 + c].i);
      }
    }
  }
}

// Occupancy target (waves per SIMD the register allocation must allow): 5
// for FP16S (96 VGPRs, no spills), 4 for FP32 (128; it would spill at 5), 3
// for FP64 (about 168); the stencil hides latency by occupancy.
template <int P>
struct HopOcc {
  static constexpr int waves = P == P64 ? 3 : (P == P16 ? kOcc16 : 4);
};

// the same-site spinor of a.y: decoded from the words prefetched with the
// last hop direction (YPRE), else loaded here
template <int P, bool YPRE, class R>
__device__ __forceinline__ void load_y(const void* y, const FD& fd, int r, int s, int site, const DirIn<P16>& pre,
                                       cx<R>* out) {
  if constexpr (YPRE) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const h2_t h = __builtin_bit_cast(h2_t, pre.w[c]);
      out[c] = {pre.sc * (R)(float)h.x, pre.sc * (R)(float)h.y};
    }
  } else {
    ld_spinor<P>(y, fd, r, s, site, out);
  }
}

__device__ void finalize_step(int mode, double sum, const CgState& S, int r, double* out);

// A CG step fused into a hop launch (work-group 0 of each right-hand-side
// block): the previous launch's nblk partial sums of right-hand side r,
// reduced by the whole work-group in a fixed order (8 independent sums per
// thread, then lanes, then waves), then finalize_step on thread 0. red: one
// double per wave.
__device__ __forceinline__ void fin_block(int mode, const double* __restrict__ pr, int nblk, const CgState& S, int r,
                                          double* red) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  for (int j0 = tid; j0 < nblk; j0 += 8 * nthr) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = j0 + k * nthr;
      if (j < nblk) acc[k] += pr[j];
    }
  }
#pragma unroll
  for (int w = 4; w > 0; w >>= 1)
#pragma unroll
    for (int k = 0; k < w; ++k) acc[k] += acc[k + w];
  double t = acc[0];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = t;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < (nthr + 63) / 64; ++w) sum += red[w];
    finalize_step(mode, sum, S, r, nullptr);
  }
  __syncthreads();
}

// RL = 16: Ls = 16, each site's s-column is one DPP row and every exchange
// along s (D~ premix, L, the dense Ls x Ls epilogues, the rank-one sums) is
// a row rotation; RL = 0: any Ls, exchanges through lane permutes and LDS;
// RL = 4: the same for Ls a multiple of 4 (FP16S), whose columns hold whole
// 4-lane blocks, so the SU(3) products can run on the matrix cores.
template <int P, int PR, int ROLE, int RL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HopOcc<P>::waves, 8)))
hop_kernel(HopArgs a) {
  using RT = RoleT<ROLE>;
  using R = typename ST<P>::R;
  using L = HopLds<R>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ double s_red[MAXW];

  const int Ls = a.Ls, Vh = a.Vh;
  const int G = sites_per_wave(Ls);
  const int W = a.W;
  const int SBk = W * G;  // 4D sites per work-group
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane / Ls;
  const int s = lane - g * Ls;
  const bool in_col = g < G;  // lanes 64 - 64 % Ls .. 63 are idle
  const int ls = min(wave * G + g, SBk - 1);
  // Work-groups are dealt round-robin to the 8 XCDs, each with its own L2:
  // give XCD x a contiguous run of tiles so the +-z, +-t neighbours a tile
  // reads were mostly fetched by the same XCD (a bijection of [0, gridDim.x)).
  const int nblk = gridDim.x, xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int tile = xcd * (nblk / 8) + min(xcd, nblk % 8) + slot;
  // the tile's sites are positions k0 .. k0+SBk-1 of the traversal order
  // (a.order: position -> checkerboard index), which visits the lattice in
  // small (y, z, t) blocks of x-rows so that the neighbours a tile reads were
  // fetched recently by the same XCD
  const int k0 = tile * SBk;
  const int kk = k0 + wave * G + g;
  const bool live = in_col && (kk < Vh);
  // the site index itself is staged in LDS (slot 8 of the neighbour row) and
  // re-read where it is used, so it occupies no register across the kernel
  const volatile int* s_self = nullptr;
  const FD fd = {Ls, Vh, a.nrhs};

  // the structured inverse (any Ls) needs no matrix in LDS
  constexpr bool SINV = RT::AM == A_DMINV || RT::AM == A_MINVDT;
  constexpr bool DENSE = RT::AM == A_MAT || RT::AM == A_MATDT;
  constexpr bool BDENSE = RT::BM == B_DENSE;  // never together with DENSE: one matrix in LDS
  unsigned char* p = smem;
  cx<R>* s_link = (cx<R>*)p;
  p += L::links(SBk);
  int* s_nbr = (int*)p;
  p += L::nbr(SBk);
  R* s_mA = (R*)p;
  if (DENSE || BDENSE) p += L::mat(Ls);
  cx<R>* s_col = (cx<R>*)p;  // SBk x (Ls*6+1) complex: one chirality half of each column
  const int cstr = Ls * 6 + 1;
  (void)s_col;

  // stage the links and neighbour indices of this block's sites
  for (int j = tid; j < SBk * 72; j += nthr) {
    const int site = j / 72, k = j - site * 72;
    if constexpr (P == P16) {  // (Re u, -Im u) and (Im u, Re u) as half2 words
      unsigned w = 0u;
      if (k0 + site < Vh) w = ((const unsigned*)a.links)[(size_t)a.order[k0 + site] * 72 + k];
      s_link[site * LSTR + k] = {__uint_as_float(w ^ 0x80000000u), __uint_as_float((w >> 16) | (w << 16))};
    } else {
      cx<R> v = {R(0), R(0)};
      if (k0 + site < Vh) v = ld_link<P>(a.links, (size_t)a.order[k0 + site] * 72 + k);
      s_link[site * LSTR + k] = v;
    }
  }
  for (int j = tid; j < SBk * 8; j += nthr) {
    const int site = j / 8, k = j - site * 8;
    s_nbr[site * NSTR + k] = (k0 + site < Vh) ? a.nbr[(size_t)a.order[k0 + site] * 8 + k] : 0;
  }
  for (int site = tid; site < SBk; site += nthr) s_nbr[site * NSTR + 8] = a.order[min(k0 + site, Vh - 1)];
  s_self = s_nbr + ls * NSTR + 8;
#define EOFA_SITE (*s_self)

  const int rb0 = blockIdx.y * a.rhs_block;
  const int rb1 = min(rb0 + a.rhs_block, a.nrhs);
  // the fused CG step of the previous launch's partial sums (K3 takes the
  // alpha step that K4 reads): only this launch's work-group 0 writes the CG
  // state; the other work-groups may read a halt flag before or after it is
  // set, and either is right (a right-hand side halted by this step is not
  // used by the next launch)
  if constexpr (ROLE == ROLE_K3 || ROLE == ROLE_D3) {  // the third launch of an iteration, either form
    if (a.fin_partial != nullptr && blockIdx.x == 0)
      for (int r = rb0; r < rb1; ++r)
        fin_block(a.fin_mode, a.fin_partial + (size_t)r * a.fin_nblk, a.fin_nblk, a.fin_S, r, s_red);
  }
  __shared__ int s_halt;
  for (int r = rb0; r < rb1; ++r) {
    __syncthreads();
    if (a.halt != nullptr) {
      // one read of the flag per work-group, broadcast through LDS: another
      // stream may set it while this kernel runs, and every wave of the
      // block must take the same branch (the epilogues hold barriers)
      if (tid == 0) s_halt = __hip_atomic_load(a.halt + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      if (s_halt != 0) continue;
    }
    if constexpr (DENSE || BDENSE) {
      const double* mats_r = a.mats + (size_t)r * NMAT * 2 * Ls * Ls;
      load_mat<R>(s_mA, mats_r + (size_t)(DENSE ? a.matA : a.matB) * 2 * Ls * Ls, Ls, tid, nthr);
    }
    __syncthreads();

    cx<R> acc[12];
    // FP16S: the same-site y of the B term arrives with the last direction
    constexpr bool YPRE = P == P16 && RT::BM != B_NONE;
    DirIn<P16> ypre;
    const R cpd = (R)a.cpd, cmd = (R)a.cmd;
    // the epilogue's leading factor, applied by the hop once per direction
    // instead of once per component: the sign of A_NEG / A_NDTT, the (c+d)
    // of D~ and D~^T (which then act as 1 + q L, q = (c-d)/(c+d)) and the
    // normalisation of the structured M_ee^-1
    R fold = R(1);
    if constexpr (RT::AM == A_NEG) fold = R(-1);
    if constexpr (RT::AM == A_DTT || RT::AM == A_MATDT || RT::AM == A_DMINV || RT::AM == A_MINVDT) fold = cpd;
    if constexpr (RT::AM == A_NDTT) fold = -cpd;
    if constexpr (SINV) fold *= minv_norm<R>((R)a.bee, (R)a.cee, (R)a.mop[r], Ls);
    // the residual update r -= alpha v takes -alpha into v itself: the hop
    // through the fold, the same-site term through its coefficients
    R vscale = R(1);
    if constexpr (RT::OM == O_RUPD) vscale = -(R)a.alpha[r];
    fold *= vscale;
    hop_site<P, RT::DAG, RT::PRE, RL, YPRE>(a, fd, r, s, g, ls, s_link, s_nbr, acc, ypre, fold);
    (void)ypre;
    // an unconditional use: stops the hop arithmetic from being sunk into the
    // (live-only) store block, away from the per-direction loads and shuffles
#pragma unroll
    for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(acc[c].r), "+v"(acc[c].i));

    // fifth-dimension neighbours in this wave
    SNbr<R> nb;
    {
      const R m = (R)a.mop[r];
      nb.sp = g * Ls + (s > 0 ? s - 1 : Ls - 1);
      nb.sn = g * Ls + (s < Ls - 1 ? s + 1 : 0);
      nb.fp = s > 0 ? R(1) : -m;
      nb.fn = s < Ls - 1 ? R(1) : -m;
    }
    const R qd = cmd * recip(cpd);  // D~ = (c+d)(1 + qd L), the (c+d) in the fold

    cx<R> v[12];
    if constexpr (RT::AM == A_ID || RT::AM == A_MAT || RT::AM == A_DMINV || RT::AM == A_NEG) {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = acc[c];
    } else if constexpr (RL == 16 && sizeof(R) == 4) {  // D~^T h in place: L_+^T = L_- and back
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = acc[c];
      scan_step<R, 1, false>(v, s, qd, (R)a.mop[r]);
      scan_step<R, 1, true>(v + 6, s, qd, (R)a.mop[r]);
    } else {  // D~^T h = (c+d)(h + qd L^T h), the (c+d) and the sign in the fold
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = acc[c];
      lacc<R, true, RL>(v, acc, nb, qd);
    }
    if constexpr (SINV) {  // v <- M_ee^-1 v or M_ee^-T v, structured along the column
      const double* scs = a.scoef + (size_t)r * (SCOEF_HEAD + 2 * Ls);
      const R a_s = (R)scs[SCOEF_HEAD + Ls + s];
      if constexpr (RL == 16)
        minv_rows<R, RT::AM == A_MINVDT, false>(v, s, g, (R)a.bee, (R)a.cee, (R)a.mop[r], (R)scs[1], (int)scs[2],
                                                a_s);
      else
        minv_cols<R, RT::AM == A_MINVDT, false>(v, s, g, Ls, (R)a.bee, (R)a.cee, (R)a.mop[r], (R)scs[1],
                                                 (int)scs[2], a_s, s_col + ls * cstr, in_col);
#pragma unroll
      for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(v[c].r), "+v"(v[c].i));
    } else if constexpr (DENSE && RL == 16) {  // v <- M v along the row's diagonals
      cx<R> src[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) src[c] = v[c];
      row_matvec<R>(s_mA, src, s, v, false);
    } else if constexpr (DENSE) {  // v <- M v through the column in LDS
      cx<R>* mycol = s_col + ls * cstr;
      cx<R> src[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) src[c] = v[c];
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        if (half == 1) __syncthreads();
        if (in_col)
          for (int c = 0; c < 6; ++c) mycol[s * 6 + c] = src[half * 6 + c];
        __syncthreads();
        col_matvec<R>(s_mA, mycol, Ls, s, half, v, false);
      }
    }
    if constexpr (RT::AM == A_DMINV && RL == 16 && sizeof(R) == 4) {  // D~ in place along the row
      scan_step<R, 1, true>(v, s, qd, (R)a.mop[r]);
      scan_step<R, 1, false>(v + 6, s, qd, (R)a.mop[r]);
    } else if constexpr (RT::AM == A_DMINV) {  // v <- D~ v = (c+d)(v + qd L v), the (c+d) in the fold
      lacc<R, false, RL>(v, v, nb, qd);
    }
    if constexpr (BDENSE && RL == 16) {  // v += M y along the row's diagonals
      cx<R> y[12];
      load_y<P, YPRE>(a.y, fd, r, s, EOFA_SITE, ypre, y);
#pragma unroll
      for (int c = 0; c < 12; ++c) y[c] = vscale * y[c];
      row_matvec<R>(s_mA, y, s, v, true);
    } else if constexpr (BDENSE) {  // v += M y, M dense per chirality, through the column in LDS
      cx<R> y[12];
      load_y<P, YPRE>(a.y, fd, r, s, EOFA_SITE, ypre, y);
#pragma unroll
      for (int c = 0; c < 12; ++c) y[c] = vscale * y[c];
      cx<R>* mycol = s_col + ls * cstr;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        if (half == 1) __syncthreads();
        if (in_col)
          for (int c = 0; c < 6; ++c) mycol[s * 6 + c] = y[half * 6 + c];
        __syncthreads();
        col_matvec<R>(s_mA, mycol, Ls, s, half, v, true);
      }
    } else if constexpr (RT::BM != B_NONE) {
      // + M_ee y (B_MEE) or + M_ee^T y (B_MEET):
      //   bee y - cee L y (L^T y) + sk u e_{s*}^T y (sk e_{s*} u^T y) on chirality chi
      cx<R> y[12];
      load_y<P, YPRE>(a.y, fd, r, s, EOFA_SITE, ypre, y);
      // B_MEE_DTI: M_ee D~^-1 y with the normalisation of D~^-1 moved onto
      // the coefficients of M_ee (bee, cee and the rank-one sk)
      R yn = R(1);
      if constexpr (RT::BM == B_MEE_DTI) {
        dtinv<R, RL, false>(y, s, g, Ls, cpd, cmd, (R)a.mop[r]);
        yn = dtinv_norm<R>(cpd, cmd, (R)a.mop[r], Ls);
      }
      const R bee = (R)a.bee * yn * vscale, cee = (R)a.cee * yn * vscale;
      if constexpr (RL == 16 && sizeof(R) == 4) {  // the L term rides on the rotation
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {fma(bee, y[c].r, v[c].r), fma(bee, y[c].i, v[c].i)};
        constexpr bool TR = RT::BM == B_MEET;  // L^T: L_+^T = L_- and back
        lacc_rows<!TR>(v, y, s, -cee, (R)a.mop[r]);
        lacc_rows<TR>(v + 6, y + 6, s, -cee, (R)a.mop[r]);
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {fma(bee, y[c].r, v[c].r), fma(bee, y[c].i, v[c].i)};
        lacc<R, RT::BM == B_MEET, RL>(v, y, nb, -cee);
      }
      const double* sc = a.scoef + (size_t)r * (SCOEF_HEAD + 2 * Ls);
      const R sk = (R)sc[1] * yn * vscale;
      if (sk != R(0)) {  // uniform over the block
        const int chi = (int)sc[2];
        const R us = (R)sc[SCOEF_HEAD + s];
        if (chi > 0)
          rank_one<R, RT::BM == B_MEET, 0, RL>(y, v, sk, us, g * Ls + Ls - 1, s == Ls - 1, s_col + ls * cstr, s,
                                           Ls, in_col);
        else
          rank_one<R, RT::BM == B_MEET, 6, RL>(y, v, sk, us, g * Ls, s == 0, s_col + ls * cstr, s, Ls, in_col);
      }
    }

    // FP16S outputs return the site's |v|^2 from their encoding (scaled by
    // the site maximum, so FP32 cannot overflow); the others sum it in FP64
    constexpr bool NRM16 = RT::NRM && ((RT::OM == O_STORE && P == P16) ||
                                       ((RT::OM == O_RUPD || RT::OM == O_STORE_R) && PR == P16));
    double nrm = 0.0;
    if (live) {
      if constexpr (RT::OM == O_STORE && NRM16) {
        nrm = st_spinor16<false>(a.out, fd, r, s, EOFA_SITE, v);
      } else if constexpr (RT::OM == O_STORE) {
        st_spinor<P>(a.out, fd, r, s, EOFA_SITE, v);
      } else if constexpr (RT::OM == O_ADDZ) {
        cx<R> z[12];
        ld_spinor<P>(a.z, fd, r, s, EOFA_SITE, z);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = z[c] - v[c];
        st_spinor<P>(a.out, fd, r, s, EOFA_SITE, v);
      } else {
        using RR = typename ST<PR>::R;
        cx<RR> w[12];
        if constexpr (RT::OM == O_RUPD && PR == P16) {
          // r + (-alpha v) from the raw half words (v carries -alpha): one
          // mixed-precision FMA per component instead of decode, scale, FMA
          float sc;
          unsigned hw[12];
          ld_raw16_nt(a.r, fd, r, s, EOFA_SITE, sc, hw);
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            const h2_t h = __builtin_bit_cast(h2_t, hw[c]);
            w[c].r = fma((float)h.x, sc, (float)v[c].r);
            w[c].i = fma((float)h.y, sc, (float)v[c].i);
          }
        } else if constexpr (RT::OM == O_RUPD) {  // r + (-alpha v), v carries -alpha
          ld_spinor_nt<PR>(a.r, fd, r, s, EOFA_SITE, w);
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            w[c].r = w[c].r + (RR)v[c].r;
            w[c].i = w[c].i + (RR)v[c].i;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 12; ++c) w[c] = {(RR)v[c].r, (RR)v[c].i};
        }
        if constexpr (NRM16)
          nrm = st_spinor16<true>(a.r, fd, r, s, EOFA_SITE, w);
        else
          st_spinor_nt<PR>(a.r, fd, r, s, EOFA_SITE, w);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {(R)w[c].r, (R)w[c].i};
      }
      if constexpr (RT::NRM && !NRM16) {
#pragma unroll
        for (int c = 0; c < 12; ++c) nrm += (double)v[c].r * v[c].r + (double)v[c].i * v[c].i;
      }
    }
    if constexpr (RT::NRM) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
      if (lane == 0) s_red[wave] = nrm;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < W; ++w) t += s_red[w];
        a.partial[(size_t)r * gridDim.x + blockIdx.x] = t;
      }
    }
  }
}

#undef EOFA_SITE

// precision of the CG residual a hop kernel updates: FP16S inner solves keep
// it in FP16S too (reliable updates replace it long before its rounding
// matters), so every field of the FP16S iteration is half width
template <int P>
constexpr int acc_prec() {
  return P;
}

int hop_blocks(int prec, int Vh, int Ls, int W) {
  (void)prec;
  const int SBk = W * sites_per_wave(Ls);
  return (Vh + SBk - 1) / SBk;
}

// the row form (RL = 16) serves Ls = 16 at every precision
template <int P>
bool use_rows(int Ls) { return Ls == 16; }

template <int P, int ROLE>
size_t hop_lds_t(int Ls, int W) {
  using R = typename ST<P>::R;
  using RT = RoleT<ROLE>;
  using L = HopLds<R>;
  const int SBk = W * sites_per_wave(Ls);
  const bool DENSE = RT::AM == A_MAT || RT::AM == A_MATDT || RT::BM == B_DENSE;
  size_t lds = L::links(SBk) + L::nbr(SBk);
  if (DENSE) lds += L::mat(Ls);
  // column slots: dense products, and the transposed rank-one sums (B_MEET,
  // the structured M_ee^-T) when the column is not a DPP row
  if ((DENSE || RT::BM == B_MEET || RT::AM == A_MINVDT) && !use_rows<P>(Ls)) lds += L::col(SBk, Ls);
  return lds;
}

template <int P>
size_t hop_lds_p(int role, int Ls, int W) {
  switch (role) {
    case ROLE_DSLASH: return hop_lds_t<P, ROLE_DSLASH>(Ls, W);
    case ROLE_DSLASH_DAG: return hop_lds_t<P, ROLE_DSLASH_DAG>(Ls, W);
    case ROLE_K1: return hop_lds_t<P, ROLE_K1>(Ls, W);
    case ROLE_K2: return hop_lds_t<P, ROLE_K2>(Ls, W);
    case ROLE_K3: return hop_lds_t<P, ROLE_K3>(Ls, W);
    case ROLE_K4: return hop_lds_t<P, ROLE_K4>(Ls, W);
    case ROLE_K4S: return hop_lds_t<P, ROLE_K4S>(Ls, W);
    case ROLE_SRC: return hop_lds_t<P, ROLE_SRC>(Ls, W);
    case ROLE_RES: return hop_lds_t<P, ROLE_RES>(Ls, W);
    case ROLE_FULLRES: return hop_lds_t<P, ROLE_FULLRES>(Ls, W);
    case ROLE_D1: return hop_lds_t<P, ROLE_D1>(Ls, W);
    case ROLE_D2: return hop_lds_t<P, ROLE_D2>(Ls, W);
    case ROLE_D3: return hop_lds_t<P, ROLE_D3>(Ls, W);
    case ROLE_D4: return hop_lds_t<P, ROLE_D4>(Ls, W);
    case ROLE_D4S: return hop_lds_t<P, ROLE_D4S>(Ls, W);
    case ROLE_DSRC: return hop_lds_t<P, ROLE_DSRC>(Ls, W);
    case ROLE_DRES: return hop_lds_t<P, ROLE_DRES>(Ls, W);
    case ROLE_DFULLRES: return hop_lds_t<P, ROLE_DFULLRES>(Ls, W);
    case ROLE_K1T: return hop_lds_t<P, ROLE_K1T>(Ls, W);
    case ROLE_K2T: return hop_lds_t<P, ROLE_K2T>(Ls, W);
  }
  return 0;
}

size_t hop_lds_bytes(int prec, int role, int Ls, int W) {
  return prec == P64 ? hop_lds_p<P64>(role, Ls, W) : prec == P32 ? hop_lds_p<P32>(role, Ls, W)
                                                                  : hop_lds_p<P16>(role, Ls, W);
}

template <int P, int ROLE>
int launch_hop_t(const HopArgs& a, hipStream_t st, int* nblk_out) {
  const int Ls = a.Ls;
  const int W = a.W >= 1 && a.W <= MAXW ? a.W : default_waves(Ls);
  const size_t lds = hop_lds_t<P, ROLE>(Ls, W);
  const int nblk = hop_blocks(P, a.Vh, Ls, W);
  const int rb = a.rhs_block > 0 ? a.rhs_block : 1;
  dim3 grid(nblk, (a.nrhs + rb - 1) / rb);
  HopArgs b = a;
  b.rhs_block = rb;
  b.W = W;
  void (*fn)(HopArgs) = hop_kernel<P, acc_prec<P>(), ROLE, 0>;
  if constexpr (P == P16)
    if (Ls % 4 == 0) fn = hop_kernel<P, acc_prec<P>(), ROLE, 4>;
  if (use_rows<P>(Ls)) fn = hop_kernel<P, acc_prec<P>(), ROLE, 16>;
  if (lds > 65536) {
    if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess)
      return EOFA_ERR_HIP;
  }
  hipLaunchKernelGGL(fn, grid, dim3(64 * W), lds, st, b);
  if (nblk_out) *nblk_out = nblk;
  return hipGetLastError() == hipSuccess ? EOFA_OK : EOFA_ERR_HIP;
}

template <int P>
int launch_hop_p(int role, const HopArgs& a, hipStream_t st, int* nb) {
  switch (role) {
    case ROLE_DSLASH: return launch_hop_t<P, ROLE_DSLASH>(a, st, nb);
    case ROLE_DSLASH_DAG: return launch_hop_t<P, ROLE_DSLASH_DAG>(a, st, nb);
    case ROLE_K1: return launch_hop_t<P, ROLE_K1>(a, st, nb);
    case ROLE_K2: return launch_hop_t<P, ROLE_K2>(a, st, nb);
    case ROLE_K3: return launch_hop_t<P, ROLE_K3>(a, st, nb);
    case ROLE_K4: return launch_hop_t<P, ROLE_K4>(a, st, nb);
    case ROLE_K4S: return launch_hop_t<P, ROLE_K4S>(a, st, nb);
    case ROLE_SRC: return launch_hop_t<P, ROLE_SRC>(a, st, nb);
    case ROLE_RES: return launch_hop_t<P, ROLE_RES>(a, st, nb);
    case ROLE_FULLRES: return launch_hop_t<P, ROLE_FULLRES>(a, st, nb);
    case ROLE_D1: return launch_hop_t<P, ROLE_D1>(a, st, nb);
    case ROLE_D2: return launch_hop_t<P, ROLE_D2>(a, st, nb);
    case ROLE_D3: return launch_hop_t<P, ROLE_D3>(a, st, nb);
    case ROLE_D4: return launch_hop_t<P, ROLE_D4>(a, st, nb);
    case ROLE_D4S: return launch_hop_t<P, ROLE_D4S>(a, st, nb);
    case ROLE_DSRC: return launch_hop_t<P, ROLE_DSRC>(a, st, nb);
    case ROLE_DRES: return launch_hop_t<P, ROLE_DRES>(a, st, nb);
    case ROLE_DFULLRES: return launch_hop_t<P, ROLE_DFULLRES>(a, st, nb);
    case ROLE_K1T: return launch_hop_t<P, ROLE_K1T>(a, st, nb);
    case ROLE_K2T: return launch_hop_t<P, ROLE_K2T>(a, st, nb);
  }
  return EOFA_ERR_INVALID;
}

int launch_hop(int prec, int role, const HopArgs& a, hipStream_t st, int* nblk_out) {
  switch (prec) {
    case P64: return launch_hop_p<P64>(role, a, st, nblk_out);
    case P32: return launch_hop_p<P32>(role, a, st, nblk_out);
    case P16: return launch_hop_p<P16>(role, a, st, nblk_out);
  }
  return EOFA_ERR_INVALID;
}

// ---------------------------------------------------------------------------
// geometry helpers

struct GeoD {
  int L[4];
  int Ls, Vh;
};

__device__ __forceinline__ void site_coords(const GeoD& g, int parity, int i, int x[4]) {
  const int hx = g.L[0] / 2;
  int rest = i / hx;
  const int xh = i - rest * hx;
  x[1] = rest % g.L[1];
  rest /= g.L[1];
  x[2] = rest % g.L[2];
  x[3] = rest / g.L[2];
  x[0] = 2 * xh + ((x[1] + x[2] + x[3] + parity) & 1);
}

__device__ __forceinline__ size_t lex(const GeoD& g, const int x[4]) {
  return (((size_t)x[3] * g.L[2] + x[2]) * g.L[1] + x[1]) * g.L[0] + x[0];
}

static GeoD geo_d(const Geometry& g) {
  GeoD d;
  for (int k = 0; k < 4; ++k) d.L[k] = g.L[k];
  d.Ls = g.Ls;
  d.Vh = g.Vh;
  return d;
}

// ---------------------------------------------------------------------------
// gauge packing: per output parity p and site i, 8 links
//   dir mu   : U_mu(x) * (bc_mu if x_mu = L_mu - 1)
//   dir 4+mu : U_mu(x - mu)^dag * (bc_mu if x_mu = 0)
// and the checkerboard index of the neighbour x +- mu (parity 1-p).

__global__ void gauge_pack_kernel(GeoD g, const double2* __restrict__ U, int bc0, int bc1, int bc2, int bc3,
                                  double2* l64p0, double2* l64p1, float2* l32p0, float2* l32p1,
                                  unsigned int* l16p0, unsigned int* l16p1, int* nbr0, int* nbr1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= g.Vh) return;
  const int bc[4] = {bc0, bc1, bc2, bc3};
  int x[4];
  site_coords(g, p, i, x);
  const size_t V = (size_t)g.L[0] * g.L[1] * g.L[2] * g.L[3];
  double2* l64 = p ? l64p1 : l64p0;
  float2* l32 = p ? l32p1 : l32p0;
  unsigned int* l16 = p ? l16p1 : l16p0;
  int* nbr = p ? nbr1 : nbr0;
  for (int dir = 0; dir < 8; ++dir) {
    const int mu = dir & 3;
    const bool fwd = dir < 4;
    int y[4] = {x[0], x[1], x[2], x[3]};
    double sign = 1.0;
    if (fwd) {
      if (x[mu] == g.L[mu] - 1) sign = bc[mu];
      y[mu] = (x[mu] + 1) % g.L[mu];
    } else {
      if (x[mu] == 0) sign = bc[mu];
      y[mu] = (x[mu] - 1 + g.L[mu]) % g.L[mu];
    }
    nbr[(size_t)i * 8 + dir] = (int)(lex(g, y) / 2);
    const size_t site = fwd ? lex(g, x) : lex(g, y);
    const double2* u = U + ((size_t)mu * V + site) * 9;
    for (int a3 = 0; a3 < 3; ++a3)
      for (int b = 0; b < 3; ++b) {
        double2 v = fwd ? u[a3 * 3 + b] : make_double2(u[b * 3 + a3].x, -u[b * 3 + a3].y);
        v.x *= sign;
        v.y *= sign;
        const size_t j = ((size_t)i * 8 + dir) * 9 + a3 * 3 + b;
        l64[j] = v;
        l32[j] = make_float2((float)v.x, (float)v.y);
        h2_t h;
        h.x = (_Float16)v.x;
        h.y = (_Float16)v.y;
        l16[j] = __builtin_bit_cast(unsigned int, h);
      }
  }
}

void launch_gauge_pack(const Geometry& g, const void* gauge, const int bc[4], void* l64[2], void* l32[2],
                       void* l16[2], int* nbr[2], hipStream_t st) {
  const GeoD d = geo_d(g);
  dim3 grid((g.Vh + 127) / 128, 2);
  hipLaunchKernelGGL(gauge_pack_kernel, grid, dim3(128), 0, st, d, (const double2*)gauge, bc[0], bc[1], bc[2],
                     bc[3], (double2*)l64[0], (double2*)l64[1], (float2*)l32[0], (float2*)l32[1],
                     (unsigned int*)l16[0], (unsigned int*)l16[1], nbr[0], nbr[1]);
}

// ---------------------------------------------------------------------------
// pack / unpack: canonical [rhs][Ls][T][Z][Y][X][4][3] complex128 <-> packed parity

template <int P>
__global__ void __launch_bounds__(256) pack_kernel(GeoD g, int parity, int nrhs, int g5r5, const double2* __restrict__ full, void* packed) {
  using R = typename ST<P>::R;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= g.Ls * g.Vh) return;
  const int i = idx / g.Ls, s = idx - i * g.Ls;
  int x[4];
  site_coords(g, parity, i, x);
  const size_t V = (size_t)g.L[0] * g.L[1] * g.L[2] * g.L[3];
  const int ssrc = g5r5 ? g.Ls - 1 - s : s;
  const double2* src = full + (((size_t)r * g.Ls + ssrc) * V + lex(g, x)) * 12;
  cx<R> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 t = src[c];
    const double sg = (g5r5 && c >= 6) ? -1.0 : 1.0;
    v[c] = {(R)(sg * t.x), (R)(sg * t.y)};
  }
  const FD f = {g.Ls, g.Vh, nrhs};
  st_spinor<P>(packed, f, r, s, i, v);
}

template <int P>
__global__ void __launch_bounds__(256) unpack_kernel(GeoD g, int parity, int nrhs, const void* packed, double2* full) {
  using R = typename ST<P>::R;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= g.Ls * g.Vh) return;
  const int i = idx / g.Ls, s = idx - i * g.Ls;
  int x[4];
  site_coords(g, parity, i, x);
  const size_t V = (size_t)g.L[0] * g.L[1] * g.L[2] * g.L[3];
  const FD f = {g.Ls, g.Vh, nrhs};
  cx<R> v[12];
  ld_spinor<P>(packed, f, r, s, i, v);
  double2* dst = full + (((size_t)r * g.Ls + s) * V + lex(g, x)) * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) dst[c] = make_double2((double)v[c].r, (double)v[c].i);
}

void launch_pack(int prec, const Geometry& g, const void* full, void* packed, int parity, int nrhs, int g5r5,
                 hipStream_t st) {
  const GeoD d = geo_d(g);
  dim3 grid((g.Ls * g.Vh + 255) / 256, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL(pack_kernel<P64>, grid, dim3(256), 0, st, d, parity, nrhs, g5r5, (const double2*)full, packed);
  else if (prec == P32)
    hipLaunchKernelGGL(pack_kernel<P32>, grid, dim3(256), 0, st, d, parity, nrhs, g5r5, (const double2*)full, packed);
  else
    hipLaunchKernelGGL(pack_kernel<P16>, grid, dim3(256), 0, st, d, parity, nrhs, g5r5, (const double2*)full, packed);
}

void launch_unpack(int prec, const Geometry& g, const void* packed, void* full, int parity, int nrhs,
                   hipStream_t st) {
  const GeoD d = geo_d(g);
  dim3 grid((g.Ls * g.Vh + 255) / 256, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL(unpack_kernel<P64>, grid, dim3(256), 0, st, d, parity, nrhs, packed, (double2*)full);
  else if (prec == P32)
    hipLaunchKernelGGL(unpack_kernel<P32>, grid, dim3(256), 0, st, d, parity, nrhs, packed, (double2*)full);
  else
    hipLaunchKernelGGL(unpack_kernel<P16>, grid, dim3(256), 0, st, d, parity, nrhs, packed, (double2*)full);
}

// ---------------------------------------------------------------------------
// site-local fifth-dimension matrix: out(s) = sum_s' M[ch][s][s'] in(s')

template <int P>
__global__ void __launch_bounds__(256) smat_kernel(int Ls, int Vh, int nrhs, const void* in, void* out, const double* mats, int mat) {
  using R = typename ST<P>::R;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  const double* M = mats + ((size_t)r * NMAT + mat) * 2 * Ls * Ls;
  cx<R> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = {R(0), R(0)};
  for (int sp = 0; sp < Ls; ++sp) {
    cx<R> t[12];
    ld_spinor<P>(in, f, r, sp, i, t);
    const R mp = (R)M[s * Ls + sp], mm = (R)M[Ls * Ls + s * Ls + sp];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = v[c] + mp * t[c];
#pragma unroll
    for (int c = 6; c < 12; ++c) v[c] = v[c] + mm * t[c];
  }
  st_spinor<P>(out, f, r, s, i, v);
}

void launch_smat(int prec, const Geometry& g, const void* in, void* out, const double* mats, int mat, int nrhs,
                 hipStream_t st) {
  dim3 grid((g.Ls * g.Vh + 255) / 256, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL(smat_kernel<P64>, grid, dim3(256), 0, st, g.Ls, g.Vh, nrhs, in, out, mats, mat);
  else if (prec == P32)
    hipLaunchKernelGGL(smat_kernel<P32>, grid, dim3(256), 0, st, g.Ls, g.Vh, nrhs, in, out, mats, mat);
  else
    hipLaunchKernelGGL(smat_kernel<P16>, grid, dim3(256), 0, st, g.Ls, g.Vh, nrhs, in, out, mats, mat);
}

// ---------------------------------------------------------------------------
// element-wise kernels over 5D sites

template <int PI, int PO>
__global__ void __launch_bounds__(256) convert_kernel(int Ls, int Vh, int nrhs, const void* in, void* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  cx<double> v[12];
  {
    using RI = typename ST<PI>::R;
    cx<RI> t[12];
    ld_spinor<PI>(in, f, r, s, i, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {(double)t[c].r, (double)t[c].i};
  }
  using RO = typename ST<PO>::R;
  cx<RO> o[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) o[c] = {(RO)v[c].r, (RO)v[c].i};
  st_spinor<PO>(out, f, r, s, i, o);
}

template <int PI>
__global__ void __launch_bounds__(256) axpy64_kernel(int Ls, int Vh, int nrhs, double* x, const void* e) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  using RI = typename ST<PI>::R;
  cx<RI> t[12];
  ld_spinor<PI>(e, f, r, s, i, t);
  cx<double> v[12];
  ld_spinor<P64>(x, f, r, s, i, v);
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = v[c] + cx<double>{(double)t[c].r, (double)t[c].i};
  st_spinor<P64>(x, f, r, s, i, v);
}

template <int P>
__global__ void __launch_bounds__(256) zero_kernel(int Ls, int Vh, int nrhs, void* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  using R = typename ST<P>::R;
  cx<R> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = {R(0), R(0)};
  st_spinor<P>(out, f, r, s, i, v);
}

__device__ __forceinline__ void block_sum_store(double v, double* dst) {
  __shared__ double red[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
    *dst = t;
  }
}

template <int P>
__global__ void __launch_bounds__(256) norm2_kernel(int Ls, int Vh, int nrhs, const void* in, double* partial) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  double n = 0.0;
  if (idx < Ls * Vh) {
    const int i = idx / Ls, s = idx - i * Ls;
    const FD f = {Ls, Vh, nrhs};
    using R = typename ST<P>::R;
    cx<R> v[12];
    ld_spinor<P>(in, f, r, s, i, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) n += (double)v[c].r * v[c].r + (double)v[c].i * v[c].i;
  }
  block_sum_store(n, partial + (size_t)r * gridDim.x + blockIdx.x);
}

// x += alpha p;  p = r + beta p   (CG, after the residual update; x in PX,
// the residual in PR)
template <int PS, int PX, int PR>
__global__ void __launch_bounds__(256) cg_update_kernel(int Ls, int Vh, int nrhs, void* x, const void* rr, void* p, const double* alpha,
                                 const double* beta, const int* u2run) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh || u2run[r] == 0) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  using RR = typename ST<PX>::R;
  using RS = typename ST<PS>::R;
  cx<RS> pv[12];
  cx<RR> xv[12], rv[12];
  ld_spinor<PS>(p, f, r, s, i, pv);  // p is re-read by the next hop's neighbours: cached
  ld_spinor_nt<PX>(x, f, r, s, i, xv);
  ld_spinor_nt<PR>(rr, f, r, s, i, rv);
  const RR al = (RR)alpha[r], be = (RR)beta[r];
  cx<RS> pn[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const cx<RR> pc = {(RR)pv[c].r, (RR)pv[c].i};
    xv[c].r = fma(al, pc.r, xv[c].r);
    xv[c].i = fma(al, pc.i, xv[c].i);
    pn[c] = {(RS)fma(be, pc.r, rv[c].r), (RS)fma(be, pc.i, rv[c].i)};
  }
  st_spinor_nt<PX>(x, f, r, s, i, xv);
  st_spinor<PS>(p, f, r, s, i, pn);
}

#define EOFA_EW_GRID dim3((g.Ls * g.Vh + 255) / 256, nrhs), dim3(256), 0, st

void launch_convert(int pin, int pout, const Geometry& g, const void* in, void* out, int nrhs, hipStream_t st) {
#define CV(A, B)                                                                          \
  if (pin == A && pout == B) {                                                            \
    hipLaunchKernelGGL((convert_kernel<A, B>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, in, out); \
    return;                                                                               \
  }
  CV(P64, P64) CV(P64, P32) CV(P64, P16) CV(P32, P64) CV(P32, P32) CV(P32, P16) CV(P16, P64) CV(P16, P32)
  CV(P16, P16)
#undef CV
}

void launch_axpy_to64(int pin, const Geometry& g, void* x64, const void* e, int nrhs, hipStream_t st) {
  if (pin == P64)
    hipLaunchKernelGGL(axpy64_kernel<P64>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, (double*)x64, e);
  else if (pin == P32)
    hipLaunchKernelGGL(axpy64_kernel<P32>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, (double*)x64, e);
  else
    hipLaunchKernelGGL(axpy64_kernel<P16>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, (double*)x64, e);
}

void launch_zero(int prec, const Geometry& g, void* f, int nrhs, hipStream_t st) {
  if (prec == P64)
    hipLaunchKernelGGL(zero_kernel<P64>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f);
  else if (prec == P32)
    hipLaunchKernelGGL(zero_kernel<P32>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f);
  else
    hipLaunchKernelGGL(zero_kernel<P16>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f);
}

int launch_norm2(int prec, const Geometry& g, const void* f, int nrhs, double* partial, hipStream_t st) {
  const int nblk = (g.Ls * g.Vh + 255) / 256;
  if (prec == P64)
    hipLaunchKernelGGL(norm2_kernel<P64>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f, partial);
  else if (prec == P32)
    hipLaunchKernelGGL(norm2_kernel<P32>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f, partial);
  else
    hipLaunchKernelGGL(norm2_kernel<P16>, EOFA_EW_GRID, g.Ls, g.Vh, nrhs, f, partial);
  return nblk;
}

// CG update with the solution update batched over a ring of directions:
// p_{k+1} = r + beta p_k goes to the next ring slot, and the step's alpha is
// kept (0 when the step did not run); a right-hand side whose CG has stopped
// carries p forward, so the last direction is always in the newest slot.
template <int PS, int PR>
__global__ void __launch_bounds__(256) p_update_kernel(int Ls, int Vh, int nrhs, const void* rr, const void* p,
                                                         void* pn, const double* alpha, const double* beta,
                                                         const int* u2run, double* ahist) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const bool run = u2run[r] != 0;
  if (idx == 0) ahist[r] = run ? alpha[r] : 0.0;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  using RR = typename ST<PR>::R;
  using RS = typename ST<PS>::R;
  cx<RS> pv[12];
  ld_spinor<PS>(p, f, r, s, i, pv);
  if (run) {
    cx<RR> rv[12];
    ld_spinor_nt<PR>(rr, f, r, s, i, rv);
    const RR be = (RR)beta[r];
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = {(RS)fma(be, (RR)pv[c].r, rv[c].r), (RS)fma(be, (RR)pv[c].i, rv[c].i)};
  }
  st_spinor<PS>(pn, f, r, s, i, pv);
}

// x += sum over nslots ring slots j of ahist[j] p_j (slots first, first+1, ...
// mod R); steps that did not run have alpha 0 and are skipped (uniform per
// right-hand side, so their directions are not read)
template <int PS, int PR>
__global__ void __launch_bounds__(256) x_flush_kernel(int Ls, int Vh, int nrhs, void* x, const char* ring,
                                                        size_t slot_bytes, int first, int nslots, int R,
                                                        const double* ahist) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (idx >= Ls * Vh) return;
  const int i = idx / Ls, s = idx - i * Ls;
  const FD f = {Ls, Vh, nrhs};
  using RR = typename ST<PR>::R;
  using RS = typename ST<PS>::R;
  cx<RR> xv[12];
  ld_spinor_nt<PR>(x, f, r, s, i, xv);
  for (int j = 0; j < nslots; ++j) {
    const int slot = (first + j) % R;
    const RR a = (RR)ahist[(size_t)slot * nrhs + r];
    if (a == RR(0)) continue;
    cx<RS> pv[12];
    ld_spinor<PS>(ring + slot * slot_bytes, f, r, s, i, pv);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      xv[c].r = fma(a, (RR)pv[c].r, xv[c].r);
      xv[c].i = fma(a, (RR)pv[c].i, xv[c].i);
    }
  }
  st_spinor_nt<PR>(x, f, r, s, i, xv);
}

// The update kernels of a direction held as p~ = D~ p: lanes hold whole
// s-columns as in the hop kernel (lane = g*Ls + s, G = 64/Ls sites per wave,
// four waves per work-group), so D~ r = (c+d) r + (c-d)(P_+ L_+ r + P_- L_- r)
// (App. A) is a lane exchange. Every lane takes part in the exchange; only
// live lanes (g < G, site in range) load and store.
template <class R, int RL>
__device__ __forceinline__ void dt_apply(cx<R>* v, int s, int g, int Ls, R cpd, R cmd, R m) {
  SNbr<R> nb;
  nb.sp = g * Ls + (s > 0 ? s - 1 : Ls - 1);
  nb.sn = g * Ls + (s < Ls - 1 ? s + 1 : 0);
  nb.fp = s > 0 ? R(1) : -m;
  nb.fn = s < Ls - 1 ? R(1) : -m;
  cx<R> t[12];
  lmul<R, false, RL>(v, t, nb);
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = {fma(cmd, t[c].r, cpd * v[c].r), fma(cmd, t[c].i, cpd * v[c].i)};
}

struct ColLane {
  int g, s, i;
  bool live;
};
__device__ __forceinline__ ColLane col_lane(int Ls, int Vh) {
  const int G = 64 / Ls, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ColLane c;
  c.g = lane / Ls;
  c.s = lane - c.g * Ls;
  c.i = (blockIdx.x * 4 + wave) * G + c.g;
  c.live = c.g < G && c.i < Vh;
  return c;
}

// p~_{k+1} = D~ r + beta p~_k into the next ring slot, alpha kept (as p_update_kernel)
template <int PS, int PR, int RL>
__global__ void __launch_bounds__(256) p_update_dt_kernel(int Ls, int Vh, int nrhs, const void* rr, const void* p,
                                                            void* pn, const double* alpha, const double* beta,
                                                            const int* u2run, double* ahist, double cpd, double cmd,
                                                            const double* mop) {
  const int r = blockIdx.y;
  const ColLane cl = col_lane(Ls, Vh);
  const bool run = u2run[r] != 0;  // uniform over the grid
  if (blockIdx.x == 0 && threadIdx.x == 0) ahist[r] = run ? alpha[r] : 0.0;
  const FD f = {Ls, Vh, nrhs};
  using RR = typename ST<PR>::R;
  using RS = typename ST<PS>::R;
  cx<RS> pv[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) pv[c] = {RS(0), RS(0)};
  if (cl.live) ld_spinor<PS>(p, f, r, cl.s, cl.i, pv);
  if (run) {
    cx<RR> rv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) rv[c] = {RR(0), RR(0)};
    if (cl.live) ld_spinor_nt<PR>(rr, f, r, cl.s, cl.i, rv);
    dt_apply<RR, RL>(rv, cl.s, cl.g, Ls, (RR)cpd, (RR)cmd, (RR)mop[r]);
    const RR be = (RR)beta[r];
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = {(RS)fma(be, (RR)pv[c].r, rv[c].r), (RS)fma(be, (RR)pv[c].i, rv[c].i)};
  }
  if (cl.live) st_spinor<PS>(pn, f, r, cl.s, cl.i, pv);
}

// x~ += alpha p~;  p~ = D~ r + beta p~   (fused form of the same update)
template <int PS, int PX, int PR, int RL>
__global__ void __launch_bounds__(256) cg_update_dt_kernel(int Ls, int Vh, int nrhs, void* x, const void* rr,
                                                             void* p, const double* alpha, const double* beta,
                                                             const int* u2run, double cpd, double cmd,
                                                             const double* mop) {
  const int r = blockIdx.y;
  if (u2run[r] == 0) return;  // uniform over the block
  const ColLane cl = col_lane(Ls, Vh);
  const FD f = {Ls, Vh, nrhs};
  using RR = typename ST<PX>::R;
  using RS = typename ST<PS>::R;
  cx<RS> pv[12];
  cx<RR> xv[12], rv[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    pv[c] = {RS(0), RS(0)};
    rv[c] = {RR(0), RR(0)};
  }
  if (cl.live) {
    ld_spinor<PS>(p, f, r, cl.s, cl.i, pv);
    ld_spinor_nt<PR>(rr, f, r, cl.s, cl.i, rv);
  }
  dt_apply<RR, RL>(rv, cl.s, cl.g, Ls, (RR)cpd, (RR)cmd, (RR)mop[r]);
  if (!cl.live) return;
  ld_spinor_nt<PX>(x, f, r, cl.s, cl.i, xv);
  const RR al = (RR)alpha[r], be = (RR)beta[r];
  cx<RS> pn[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const cx<RR> pc = {(RR)pv[c].r, (RR)pv[c].i};
    xv[c].r = fma(al, pc.r, xv[c].r);
    xv[c].i = fma(al, pc.i, xv[c].i);
    pn[c] = {(RS)fma(be, pc.r, rv[c].r), (RS)fma(be, pc.i, rv[c].i)};
  }
  st_spinor_nt<PX>(x, f, r, cl.s, cl.i, xv);
  st_spinor<PS>(p, f, r, cl.s, cl.i, pn);
}

template <int PS, int PR>
void launch_p_update_dt(const Geometry& g, const void* r, const void* p, void* pn, const double* alpha,
                        const double* beta, const int* u2run, double* ahist, int nrhs, const DtArgs& dt,
                        hipStream_t st) {
  const int G = 64 / g.Ls;
  dim3 grid((g.Vh + 4 * G - 1) / (4 * G), nrhs);
  auto fn = g.Ls == 16 ? p_update_dt_kernel<PS, PR, 16> : p_update_dt_kernel<PS, PR, 0>;
  hipLaunchKernelGGL(fn, grid, dim3(256), 0, st, g.Ls, g.Vh, nrhs, r, p, pn, alpha, beta, u2run, ahist, dt.cpd,
                     dt.cmd, dt.mop);
}

template <int PS, int PX, int PR>
void launch_cg_update_dt(const Geometry& g, void* x, const void* r, void* p, const double* alpha,
                         const double* beta, const int* u2run, int nrhs, const DtArgs& dt, hipStream_t st) {
  const int G = 64 / g.Ls;
  dim3 grid((g.Vh + 4 * G - 1) / (4 * G), nrhs);
  auto fn = g.Ls == 16 ? cg_update_dt_kernel<PS, PX, PR, 16> : cg_update_dt_kernel<PS, PX, PR, 0>;
  hipLaunchKernelGGL(fn, grid, dim3(256), 0, st, g.Ls, g.Vh, nrhs, x, r, p, alpha, beta, u2run, dt.cpd, dt.cmd,
                     dt.mop);
}

void launch_p_update(int ps, const Geometry& g, const void* r, const void* p, void* pn, const double* alpha,
                     const double* beta, const int* u2run, double* ahist, int nrhs, const DtArgs& dt,
                     hipStream_t st) {
  if (dt.mop) {
    if (ps == P64)
      launch_p_update_dt<P64, P64>(g, r, p, pn, alpha, beta, u2run, ahist, nrhs, dt, st);
    else if (ps == P32)
      launch_p_update_dt<P32, P32>(g, r, p, pn, alpha, beta, u2run, ahist, nrhs, dt, st);
    else
      launch_p_update_dt<P16, P16>(g, r, p, pn, alpha, beta, u2run, ahist, nrhs, dt, st);
    return;
  }
  if (ps == P64)
    hipLaunchKernelGGL((p_update_kernel<P64, P64>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, r, p, pn, alpha, beta, u2run,
                       ahist);
  else if (ps == P32)
    hipLaunchKernelGGL((p_update_kernel<P32, P32>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, r, p, pn, alpha, beta, u2run,
                       ahist);
  else
    hipLaunchKernelGGL((p_update_kernel<P16, P16>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, r, p, pn, alpha, beta, u2run,
                       ahist);
}

void launch_x_flush(int ps, const Geometry& g, void* x, const void* ring, size_t slot_bytes, int first, int nslots,
                    int R, const double* ahist, int nrhs, hipStream_t st) {
  const char* rg = (const char*)ring;
  if (ps == P64)
    hipLaunchKernelGGL((x_flush_kernel<P64, P64>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, rg, slot_bytes, first, nslots,
                       R, ahist);
  else if (ps == P32)
    hipLaunchKernelGGL((x_flush_kernel<P32, P32>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, rg, slot_bytes, first, nslots,
                       R, ahist);
  else
    hipLaunchKernelGGL((x_flush_kernel<P16, P32>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, rg, slot_bytes, first, nslots,
                       R, ahist);
}

void launch_cg_update(int ps, const Geometry& g, void* x, const void* r, void* p, const double* alpha,
                      const double* beta, const int* u2run, int nrhs, const DtArgs& dt, hipStream_t st) {
  if (dt.mop) {
    if (ps == P64)
      launch_cg_update_dt<P64, P64, P64>(g, x, r, p, alpha, beta, u2run, nrhs, dt, st);
    else if (ps == P32)
      launch_cg_update_dt<P32, P32, P32>(g, x, r, p, alpha, beta, u2run, nrhs, dt, st);
    else
      launch_cg_update_dt<P16, P32, P16>(g, x, r, p, alpha, beta, u2run, nrhs, dt, st);
    return;
  }
  if (ps == P64)
    hipLaunchKernelGGL((cg_update_kernel<P64, P64, P64>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, r, p, alpha, beta,
                       u2run);
  else if (ps == P32)
    hipLaunchKernelGGL((cg_update_kernel<P32, P32, P32>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, r, p, alpha, beta,
                       u2run);
  else
    hipLaunchKernelGGL((cg_update_kernel<P16, P32, P16>), EOFA_EW_GRID, g.Ls, g.Vh, nrhs, x, r, p, alpha, beta,
                       u2run);
}
#undef EOFA_EW_GRID

// ---------------------------------------------------------------------------
// CG scalar finalisation: one block per right-hand side, fixed summation order

// one CG scalar step for right-hand side r from the reduced sum
__device__ void finalize_step(int mode, double sum, const CgState& S, int r, double* out) {
  if (mode == FIN_NORM) {
    out[r] = sum;
    return;
  }
  if (mode == FIN_INIT) {
    S.rr[r] = sum;
    S.stop[r] = S.tol2[r] * sum;
    S.guard[r] *= sum;
    S.iter[r] = 0;
    S.u2run[r] = 0;
    S.breakdown[r] = 0;
    S.halt[r] = (sum == 0.0 || S.max_iter[r] <= 0) ? 1 : 0;
    if (!isfinite(sum)) {
      S.breakdown[r] = 1;
      S.halt[r] = 1;
    }
    return;
  }
  if (mode == FIN_ALPHA) {
    if (S.halt[r]) return;
    S.ww[r] = sum;
    if (!(sum > 0.0) || !isfinite(sum)) {
      S.breakdown[r] = 1;
      S.halt[r] = 1;
      S.alpha[r] = 0.0;
      return;
    }
    S.alpha[r] = S.rr[r] / sum;
    return;
  }
  // FIN_BETA
  if (S.halt[r]) {
    S.u2run[r] = 0;
    return;
  }
  const double rrn = sum;
  S.beta[r] = rrn / S.rr[r];
  S.rr[r] = rrn;
  S.iter[r] += 1;
  S.u2run[r] = 1;
  if (!isfinite(rrn)) {
    S.breakdown[r] = 1;
    S.halt[r] = 1;
    S.u2run[r] = 0;
  } else if (rrn <= S.stop[r] || S.iter[r] >= S.max_iter[r]) {
    S.halt[r] = 1;
  } else if (S.guard[r] > 0.0 && rrn > S.guard[r]) {
    S.halt[r] = 1;
    S.breakdown[r] = 2;
  }
}

constexpr int FIN_THREADS = 1024, FIN_LOADS = 16;

__global__ void __launch_bounds__(FIN_THREADS) finalize_kernel(int mode, const double* __restrict__ partial,
                                                                 int nblk, CgState S, double* out) {
  const int r = blockIdx.x;
  __shared__ double red[FIN_THREADS / 64];
  // FIN_LOADS independent partial sums per thread: at the usual partial counts
  // (one per hop work-group, 16384 at 16^3 x 32 x 16) every load of the block
  // is in flight at once, so the sum costs one memory latency, not several
  const double* pr = partial + (size_t)r * nblk;
  double acc[FIN_LOADS];
#pragma unroll
  for (int k = 0; k < FIN_LOADS; ++k) acc[k] = 0.0;
  for (int j0 = threadIdx.x; j0 < nblk; j0 += FIN_LOADS * FIN_THREADS) {
#pragma unroll
    for (int k = 0; k < FIN_LOADS; ++k) {
      const int j = j0 + k * FIN_THREADS;
      if (j < nblk) acc[k] += pr[j];
    }
  }
#pragma unroll
  for (int w = FIN_LOADS / 2; w > 0; w >>= 1)
#pragma unroll
    for (int k = 0; k < w; ++k) acc[k] += acc[k + w];
  double t = acc[0];
  // per wave by lane exchange, then the wave sums in a fixed order
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < FIN_THREADS / 64; ++w) sum += red[w];
    finalize_step(mode, sum, S, r, out);
  }
}

void launch_finalize(int mode, const double* partial, int nblk, int nrhs, CgState s, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(FIN_THREADS), 0, st, mode, partial, nblk, s, out);
}

// ---------------------------------------------------------------------------
// heatbath right-hand sides and combination (canonical layout)

__global__ void omega_rhs_kernel(int Ls, size_t V, const double2* __restrict__ eta, double2* rhs,
                                 const double* om, const int* chir) {
  const size_t site = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y, r = blockIdx.z;
  if (site >= V) return;
  const double w = om[r * Ls + s];
  const int ch = chir[r];
  const double2* src = eta + site * 12;  // s = 0 slice
  double2* dst = rhs + (((size_t)r * Ls + s) * V + site) * 12;
  for (int c = 0; c < 12; ++c) {
    const bool keep = (ch > 0) ? (c < 6) : (c >= 6);
    const double2 v = src[c];
    dst[c] = keep ? make_double2(w * v.x, w * v.y) : make_double2(0.0, 0.0);
  }
}

__global__ void heatbath_combine_kernel(int Ls, size_t V, int nsys, const double2* __restrict__ eta,
                                        const double2* __restrict__ sol, double2* phi, double a_eta,
                                        const double* coef, const double* om, const int* chir) {
  const size_t site = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (site >= V) return;
  const double2* e = eta + ((size_t)s * V + site) * 12;
  double2 acc[12];
  for (int c = 0; c < 12; ++c) acc[c] = make_double2(a_eta * e[c].x, a_eta * e[c].y);
  if (s == 0) {
    for (int r = 0; r < nsys; ++r) {
      const int ch = chir[r];
      const double cf = coef[r];
      for (int sp = 0; sp < Ls; ++sp) {
        const double w = cf * om[r * Ls + sp];
        const double2* y = sol + (((size_t)r * Ls + sp) * V + site) * 12;
        for (int c = 0; c < 12; ++c) {
          const bool keep = (ch > 0) ? (c < 6) : (c >= 6);
          if (keep) {
            acc[c].x += w * y[c].x;
            acc[c].y += w * y[c].y;
          }
        }
      }
    }
  }
  double2* o = phi + ((size_t)s * V + site) * 12;
  for (int c = 0; c < 12; ++c) o[c] = acc[c];
}

void launch_omega_rhs(const Geometry& g, const void* eta, void* rhs, const double* om, const int* chir, int nsys,
                      hipStream_t st) {
  dim3 grid((g.V + 127) / 128, g.Ls, nsys);
  hipLaunchKernelGGL(omega_rhs_kernel, grid, dim3(128), 0, st, g.Ls, (size_t)g.V, (const double2*)eta,
                     (double2*)rhs, om, chir);
}

void launch_heatbath_combine(const Geometry& g, const void* eta, const void* sol, void* phi, double a_eta,
                             const double* coef, const double* om, const int* chir, int nsys, hipStream_t st) {
  dim3 grid((g.V + 127) / 128, g.Ls);
  hipLaunchKernelGGL(heatbath_combine_kernel, grid, dim3(128), 0, st, g.Ls, (size_t)g.V, nsys,
                     (const double2*)eta, (const double2*)sol, (double2*)phi, a_eta, coef, om, chir);
}

size_t packed_bytes(int prec, const Geometry& g, int nrhs) {
  const size_t n = (size_t)nrhs * 6 * g.Ls * g.Vh;
  if (prec == P64) return n * 32;
  if (prec == P32) return n * 16;
  return n * 8 + (size_t)nrhs * g.Ls * g.Vh * 4;
}

size_t link_bytes(int prec, const Geometry& g) {
  const size_t n = (size_t)g.Vh * 72;
  return n * (prec == P64 ? 16 : prec == P32 ? 8 : 4);
}

}  // namespace eofa
