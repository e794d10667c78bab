// Host FP64 set-up of the fifth-dimension matrices of one EOFA system.
//
// For operator mass m_op, shift (beta, chi) and shift masses (m_a, m_b):
//   L_+(m)  : (L_+)_{s,s-1} = 1 (s >= 1), (L_+)_{0,Ls-1} = -m;  L_- = L_+^T   (Sec. II)
//   D~_+-   = (c+d) 1 + (c-d) L_+-(m_op)                                   (eqn eofa_dop_def)
//   M_ee,+- = bee 1 - cee L_+-(m_op),  bee = (c+d)(4-M5)+1, cee = 1-(c-d)(4-M5)
//             (the site-local part of eqn Ddwf), plus chi beta u_chi v_chi^T
//             on the chirality chi (App. B.2, eqns precond_mobius_eofa_system
//             and delta_rank_one: Delta~ = R5 Delta D~ = u (x) v)
//   u_+     = (-1)^s (c-d)^s / (c+d)^(Ls+s+1) N(m_op)
//   u_-     = (-1)^(s+1) (c-d)^(Ls-1-s) / (c+d)^(2Ls-s) N(m_op),  N(m) = (c+d)^Ls + m (c-d)^Ls
//   v_+     = k e_{Ls-1},  v_- = k e_0,  k = 2c(m_b-m_a)(c+d)^(2Ls) / (N(m_a) N(m_b))  (App. A)
//   M_ee^-1 = A^-1 - sigma (A^-1 u)(v^T A^-1) / (1 + sigma v^T A^-1 u),  sigma = chi beta,
//             A = unshifted block, inverted by LU with partial pivoting
//             (eqn sherman_morrison_mobius_inv, generic form).
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace eofa {

namespace {

using Mat = std::vector<double>;  // row-major Ls x Ls

Mat eye(int n) {
  Mat a(n * n, 0.0);
  for (int i = 0; i < n; ++i) a[i * n + i] = 1.0;
  return a;
}

Mat lmat(int n, double m, int chir) {
  Mat a(n * n, 0.0);
  for (int s = 1; s < n; ++s) a[s * n + (s - 1)] = 1.0;
  a[0 * n + (n - 1)] = -m;
  if (chir < 0) {  // transpose
    Mat t(n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) t[i * n + j] = a[j * n + i];
    return t;
  }
  return a;
}

Mat transpose(const Mat& a, int n) {
  Mat t(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t[i * n + j] = a[j * n + i];
  return t;
}

Mat matmul(const Mat& a, const Mat& b, int n) {
  Mat c(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double aik = a[i * n + k];
      for (int j = 0; j < n; ++j) c[i * n + j] += aik * b[k * n + j];
    }
  return c;
}

// Inverse by Gauss-Jordan elimination with partial pivoting; false if singular.
bool invert(Mat a, int n, Mat& inv) {
  inv = eye(n);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(a[r * n + col]) > std::fabs(a[piv * n + col])) piv = r;
    if (!(std::fabs(a[piv * n + col]) > 0.0)) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(a[piv * n + j], a[col * n + j]);
        std::swap(inv[piv * n + j], inv[col * n + j]);
      }
    const double d = 1.0 / a[col * n + col];
    for (int j = 0; j < n; ++j) {
      a[col * n + j] *= d;
      inv[col * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = a[r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[r * n + j] -= f * a[col * n + j];
        inv[r * n + j] -= f * inv[col * n + j];
      }
    }
  }
  return true;
}

double sgn(int n) { return (n % 2 != 0) ? -1.0 : 1.0; }

}  // namespace

double k_eofa(int Ls, double c, double d, double m_a, double m_b);

void build_struct(const Geometry& g, double M5, double b5, double c5, const eofa_system& sys, double* out) {
  const int n = g.Ls;
  const double c = 0.5 * (b5 + c5), d = 0.5 * (b5 - c5);
  const double Nop = std::pow(c + d, n) + sys.m_op * std::pow(c - d, n);
  const bool shifted = sys.beta != 0.0;
  const int chir = shifted ? sys.chi : 1;
  out[0] = sys.m_op;
  out[1] = shifted ? chir * sys.beta * k_eofa(n, c, d, sys.m_a, sys.m_b) : 0.0;
  out[2] = chir;
  out[3] = 0.0;
  for (int s = 0; s < n; ++s) {
    if (chir > 0)
      out[SCOEF_HEAD + s] = sgn(s) * std::pow(c - d, s) / std::pow(c + d, n + s + 1) * Nop;
    else
      out[SCOEF_HEAD + s] = sgn(s + 1) * std::pow(c - d, n - 1 - s) / std::pow(c + d, 2 * n - s) * Nop;
  }
  // Sherman-Morrison column a (zero when unshifted or A is singular: the
  // dense matrices of build_fifth report that case as a breakdown)
  double* a = out + SCOEF_HEAD + n;
  for (int s = 0; s < n; ++s) a[s] = 0.0;
  if (out[1] == 0.0) return;
  const double bee = (c + d) * (4.0 - M5) + 1.0, cee = 1.0 - (c - d) * (4.0 - M5);
  Mat A(n * n, 0.0), Ainv;
  for (int s = 0; s < n; ++s) {
    A[s * n + s] = bee;
    if (chir > 0)  // L_+: (L y)_s = y_{s-1}, -m y_{Ls-1} at s = 0
      A[s * n + (s > 0 ? s - 1 : n - 1)] -= cee * (s > 0 ? 1.0 : -sys.m_op);
    else  // L_-: (L y)_s = y_{s+1}, -m y_0 at s = Ls-1
      A[s * n + (s < n - 1 ? s + 1 : 0)] -= cee * (s < n - 1 ? 1.0 : -sys.m_op);
  }
  if (!invert(A, n, Ainv)) return;
  std::vector<double> x(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) x[i] += Ainv[i * n + j] * out[SCOEF_HEAD + j];
  const int star = chir > 0 ? n - 1 : 0;
  const double den = 1.0 + out[1] * x[star];
  if (!std::isfinite(den) || std::fabs(den) < 1e-14) return;
  for (int s = 0; s < n; ++s) a[s] = -out[1] * x[s] / den;
}

double k_eofa(int Ls, double c, double d, double m_a, double m_b) {
  const double Na = std::pow(c + d, Ls) + m_a * std::pow(c - d, Ls);
  const double Nb = std::pow(c + d, Ls) + m_b * std::pow(c - d, Ls);
  return 2.0 * c * (m_b - m_a) * std::pow(c + d, 2 * Ls) / (Na * Nb);
}

void omega_col(int Ls, double c, double d, int chir, double* w) {
  for (int s = 0; s < Ls; ++s) {
    if (chir > 0)
      w[s] = sgn(s + 1) * std::pow(c - d, Ls - s - 1) / std::pow(c + d, Ls - s);
    else
      w[s] = sgn(s) * std::pow(c - d, s) / std::pow(c + d, s + 1);
  }
}

int build_fifth(const Geometry& g, double M5, double b5, double c5, const eofa_system& sys,
                double* out, std::string& err) {
  const int n = g.Ls;
  const double c = 0.5 * (b5 + c5), d = 0.5 * (b5 - c5);
  const double bee = (c + d) * (4.0 - M5) + 1.0;
  const double cee = 1.0 - (c - d) * (4.0 - M5);
  const double Nop = std::pow(c + d, n) + sys.m_op * std::pow(c - d, n);
  const bool shifted = sys.beta != 0.0;
  if (shifted && sys.chi != 1 && sys.chi != -1) {
    err = "eofa_system.chi must be +1 or -1";
    return EOFA_ERR_INVALID;
  }
  const double k = shifted ? k_eofa(n, c, d, sys.m_a, sys.m_b) : 0.0;
  for (int ci = 0; ci < 2; ++ci) {
    const int chir = ci == 0 ? +1 : -1;
    const Mat L = lmat(n, sys.m_op, chir);
    Mat Dt(n * n), A(n * n);
    for (int i = 0; i < n * n; ++i) {
      Dt[i] = (c + d) * (i % (n + 1) == 0 ? 1.0 : 0.0) + (c - d) * L[i];
      A[i] = bee * (i % (n + 1) == 0 ? 1.0 : 0.0) - cee * L[i];
    }
    Mat Ainv;
    if (!invert(A, n, Ainv)) {
      err = "same-parity block is singular";
      return EOFA_ERR_BREAKDOWN;
    }
    Mat Mee = A, Minv = Ainv;
    if (shifted && sys.chi == chir) {
      std::vector<double> u(n), v(n, 0.0);
      for (int s = 0; s < n; ++s) {
        if (chir > 0)
          u[s] = sgn(s) * std::pow(c - d, s) / std::pow(c + d, n + s + 1) * Nop;
        else
          u[s] = sgn(s + 1) * std::pow(c - d, n - 1 - s) / std::pow(c + d, 2 * n - s) * Nop;
      }
      v[chir > 0 ? n - 1 : 0] = k;
      const double sigma = chir * sys.beta;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Mee[i * n + j] += sigma * u[i] * v[j];
      std::vector<double> x(n, 0.0), vA(n, 0.0);  // x = A^-1 u, vA = v^T A^-1
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          x[i] += Ainv[i * n + j] * u[j];
          vA[j] += v[i] * Ainv[i * n + j];
        }
      double vx = 0.0;
      for (int i = 0; i < n; ++i) vx += v[i] * x[i];
      const double den = 1.0 + sigma * vx;
      if (!std::isfinite(den) || std::fabs(den) < 1e-14) {
        err = "Sherman-Morrison denominator 1 + chi beta v.x vanishes";
        return EOFA_ERR_BREAKDOWN;
      }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Minv[i * n + j] -= sigma * x[i] * vA[j] / den;
    }
    Mat Dinv;
    if (!invert(Dt, n, Dinv)) {
      err = "D~(m_op) is singular";
      return EOFA_ERR_BREAKDOWN;
    }
    const Mat DtT = transpose(Dt, n);
    const Mat MinvT = transpose(Minv, n);
    Mat mats[NMAT];
    mats[MAT_MEE] = Mee;
    mats[MAT_MEE_INV] = Minv;
    mats[MAT_MEE_T] = transpose(Mee, n);
    mats[MAT_MEE_INV_T] = MinvT;
    mats[MAT_MEE_INV_T_DT_T] = matmul(MinvT, DtT, n);
    mats[MAT_NEG_DT_T] = DtT;
    for (auto& v : mats[MAT_NEG_DT_T]) v = -v;
    mats[MAT_DT_T] = DtT;
    mats[MAT_DT] = Dt;
    mats[MAT_DT_INV] = Dinv;
    mats[MAT_DEE] = matmul(Mee, Dinv, n);
    mats[MAT_DEE_INV] = matmul(Dt, Minv, n);
    mats[MAT_DEE_T] = transpose(mats[MAT_DEE], n);
    mats[MAT_DEE_INV_T] = transpose(mats[MAT_DEE_INV], n);
    for (int m = 0; m < NMAT; ++m)
      std::memcpy(out + ((size_t)m * 2 + ci) * n * n, mats[m].data(), sizeof(double) * n * n);
  }
  for (int i = 0; i < NMAT * 2 * n * n; ++i)
    if (!std::isfinite(out[i])) {
      err = "non-finite fifth-dimension coefficient";
      return EOFA_ERR_BREAKDOWN;
    }
  return EOFA_OK;
}

// x-rows (y, z, t) in blocks of by x bz x bt rows (4 where the extent allows,
// else 2 or 1), blocks in lexicographic order (y fastest), rows inside a block
// likewise; each row contributes its Lx/2 sites of one parity in x order.
void site_order(const Geometry& g, int* out) {
  auto blk = [](int L) { return L % 4 == 0 ? 4 : (L % 2 == 0 ? 2 : 1); };
  const int Lxh = g.L[0] / 2, Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int by = blk(Ly), bz = blk(Lz), bt = blk(Lt);
  size_t k = 0;
  for (int tc = 0; tc < Lt / bt; ++tc)
    for (int zc = 0; zc < Lz / bz; ++zc)
      for (int yc = 0; yc < Ly / by; ++yc)
        for (int tt = 0; tt < bt; ++tt)
          for (int zz = 0; zz < bz; ++zz)
            for (int yy = 0; yy < by; ++yy) {
              const int t = tc * bt + tt, z = zc * bz + zz, y = yc * by + yy;
              const int row = (t * Lz + z) * Ly + y;
              for (int xh = 0; xh < Lxh; ++xh) out[k++] = row * Lxh + xh;
            }
}

}  // namespace eofa
