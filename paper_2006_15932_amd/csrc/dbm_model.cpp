// dbm_model.cpp -- host-side model tables of libdbm (FP64, computed once).
//
// For each species: the D2V16 velocity set of Eq.(15), the 16x16 moment
// matrix M whose rows are listed after Eq.(14) (row 9 read as
// (v^2+eta^2) v_y: the printed v_x repeats row 8 and makes M singular), its
// inverse by LU factorisation with partial pivoting, the 1-norm condition
// number, and the symmetry blocks used by the one-pass kernels.
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/dbm.h"
#include "dbm_internal.hpp"

namespace dbm {

namespace {

// Unit directions of the four groups (Eq.15), counter-clockwise.
const int kAxisDir[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
const int kDiagDir[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};

// In-place LU factorisation with partial pivoting, then inverse by solving
// A X = I column by column.  Returns false when a pivot is below
// rel_tol * max|A| (numerically rank-deficient).
bool lu_invert(const double *A, double *Ainv, int n, double rel_tol) {
  double lu[kNV * kNV];
  int perm[kNV];
  double amax = 0.0;
  for (int k = 0; k < n * n; ++k) {
    lu[k] = A[k];
    amax = std::fmax(amax, std::fabs(A[k]));
  }
  for (int r = 0; r < n; ++r) perm[r] = r;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(lu[r * n + k]) > std::fabs(lu[p * n + k])) p = r;
    if (!(std::fabs(lu[p * n + k]) > rel_tol * amax)) return false;
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(lu[k * n + c], lu[p * n + c]);
      std::swap(perm[k], perm[p]);
    }
    for (int r = k + 1; r < n; ++r) {
      double l = lu[r * n + k] / lu[k * n + k];
      lu[r * n + k] = l;
      for (int c = k + 1; c < n; ++c) lu[r * n + c] -= l * lu[k * n + c];
    }
  }
  for (int col = 0; col < n; ++col) {
    double y[kNV];
    for (int r = 0; r < n; ++r) {  // L y = P e_col
      double s = (perm[r] == col) ? 1.0 : 0.0;
      for (int c = 0; c < r; ++c) s -= lu[r * n + c] * y[c];
      y[r] = s;
    }
    for (int r = n - 1; r >= 0; --r) {  // U x = y
      double s = y[r];
      for (int c = r + 1; c < n; ++c) s -= lu[r * n + c] * Ainv[c * n + col];
      Ainv[r * n + col] = s / lu[r * n + r];
    }
  }
  return true;
}

double norm_1(const double *A, int n) {
  double best = 0.0;
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += std::fabs(A[r * n + c]);
    best = std::fmax(best, s);
  }
  return best;
}

// Dense reconstruction of f^eq from a 16-vector of moments through the
// symmetry blocks, exactly as the kernels do it; used to self-check the blocks
// against the dense inverse.
void block_project(const SpeciesDev &sp, const double *g, double *f) {
  const double rA[4] = {g[0], g[3], g[4] + g[6], g[13] + g[15]};
  const double rB1[2] = {g[4] - g[6], g[13] - g[15]};
  const double rB2[2] = {g[5], g[14]};
  const double rX[4] = {g[1], g[7], g[9], g[11]};
  const double rY[4] = {g[2], g[8], g[12], g[10]};
  double al[4], xi[4], ps[4], be[4];
  for (int a = 0; a < 4; ++a) {
    al[a] = xi[a] = ps[a] = 0.0;
    for (int j = 0; j < 4; ++j) {
      al[a] += sp.KA[a * 4 + j] * rA[j];
      xi[a] += sp.KE[a * 4 + j] * rX[j];
      ps[a] += sp.KE[a * 4 + j] * rY[j];
    }
  }
  be[0] = sp.KB1[0] * rB1[0] + sp.KB1[1] * rB1[1];
  be[2] = sp.KB1[2] * rB1[0] + sp.KB1[3] * rB1[1];
  be[1] = sp.KB2[0] * rB2[0] + sp.KB2[1] * rB2[1];
  be[3] = sp.KB2[2] * rB2[0] + sp.KB2[3] * rB2[1];
  for (int gi = 0; gi < 4; ++gi) {
    double p = al[gi] + be[gi], m = al[gi] - be[gi];
    double *o = f + 4 * gi;
    if (gi % 2 == 0) {
      o[0] = p + xi[gi]; o[1] = m + ps[gi]; o[2] = p - xi[gi]; o[3] = m - ps[gi];
    } else {
      double s = xi[gi] + ps[gi], d = xi[gi] - ps[gi];
      o[0] = p + s; o[1] = m - d; o[2] = p - s; o[3] = m + d;
    }
  }
}

}  // namespace

// Build the device tables of one species.  Returns DBM_OK, DBM_ERR_ARG or
// DBM_ERR_SINGULAR_M with a message in err.
int build_species(const dbm_species &in, const dbm_config &cfg, SpeciesDev &sp,
                  std::string &err) {
  std::memset(&sp, 0, sizeof(sp));
  if (!(in.m > 0) || !(in.tau > 0) || !(in.I >= 0) || !std::isfinite(in.a_stoich)) {
    err = "species needs m > 0, tau > 0, I >= 0";
    return DBM_ERR_ARG;
  }
  for (int g = 0; g < 4; ++g)
    if (!std::isfinite(in.v[g]) || !std::isfinite(in.eta[g])) {
      err = "non-finite velocity parameter";
      return DBM_ERR_ARG;
    }
  sp.m = in.m;
  sp.K = 2.0 + in.I;
  sp.tau = in.tau;
  sp.a = in.a_stoich;
  sp.inv_m = 1.0 / in.m;
  sp.inv_neg_a = in.a_stoich < 0 ? -1.0 / in.a_stoich : 0.0;
  sp.inv_K = 1.0 / sp.K;
  sp.omega = cfg.dt / in.tau;
  double vx[kNV], vy[kNV], et[kNV];
  for (int g = 0; g < 4; ++g) {
    const bool axis = (g % 2 == 0);
    sp.vg[g] = in.v[g];
    sp.qg[g] = (axis ? 1.0 : 2.0) * in.v[g] * in.v[g] + in.eta[g] * in.eta[g];
    sp.cgx[g] = cfg.dt * in.v[g] / cfg.dx;
    sp.cgy[g] = cfg.dt * in.v[g] / cfg.dy;
    for (int k = 0; k < 4; ++k) {
      const int *d = axis ? kAxisDir[k] : kDiagDir[k];
      vx[4 * g + k] = in.v[g] * d[0];
      vy[4 * g + k] = in.v[g] * d[1];
      et[4 * g + k] = in.eta[g];
    }
  }
  // Moment matrix, rows listed after Eq.(14).
  for (int i = 0; i < kNV; ++i) {
    const double x = vx[i], y = vy[i], q = x * x + y * y + et[i] * et[i];
    const double rows[kNV] = {1.0,       x,         y,         q,     x * x, x * y,
                              y * y,     q * x,     q * y,     x * x * x,    x * x * y,
                              x * y * y, y * y * y, q * x * x, q * x * y,    q * y * y};
    for (int r = 0; r < kNV; ++r) sp.M[r * kNV + i] = rows[r];
  }
  if (!lu_invert(sp.M, sp.Minv, kNV, 1e-13)) {
    err = "moment matrix is singular for these velocity parameters";
    return DBM_ERR_SINGULAR_M;
  }
  const double cond = norm_1(sp.M, kNV) * norm_1(sp.Minv, kNV);
  if (!(cond <= 1e12)) {
    err = "moment matrix condition number exceeds 1e12";
    return DBM_ERR_SINGULAR_M;
  }
  double resid = 0.0;
  for (int r = 0; r < kNV; ++r)
    for (int c = 0; c < kNV; ++c) {
      double s = 0.0;
      for (int k = 0; k < kNV; ++k) s += sp.M[r * kNV + k] * sp.Minv[k * kNV + c];
      resid = std::fmax(resid, std::fabs(s - (r == c ? 1.0 : 0.0)));
    }
  if (!(resid <= 1e-9)) {
    err = "M * M^-1 differs from the identity by more than 1e-9";
    return DBM_ERR_SINGULAR_M;
  }

  // Symmetry blocks (see SpeciesDev).
  const double *v = sp.vg, *q = sp.qg;
  const double mA[16] = {1.0,
                         1.0,
                         1.0,
                         1.0,
                         q[0],
                         q[1],
                         q[2],
                         q[3],
                         v[0] * v[0],
                         2.0 * v[1] * v[1],
                         v[2] * v[2],
                         2.0 * v[3] * v[3],
                         q[0] * v[0] * v[0],
                         2.0 * q[1] * v[1] * v[1],
                         q[2] * v[2] * v[2],
                         2.0 * q[3] * v[3] * v[3]};
  const double mB1[4] = {v[0] * v[0], v[2] * v[2], q[0] * v[0] * v[0], q[2] * v[2] * v[2]};
  const double mB2[4] = {v[1] * v[1], v[3] * v[3], q[1] * v[1] * v[1], q[3] * v[3] * v[3]};
  const double mE[16] = {v[0],
                         v[1],
                         v[2],
                         v[3],
                         q[0] * v[0],
                         q[1] * v[1],
                         q[2] * v[2],
                         q[3] * v[3],
                         v[0] * v[0] * v[0],
                         v[1] * v[1] * v[1],
                         v[2] * v[2] * v[2],
                         v[3] * v[3] * v[3],
                         0.0,
                         v[1] * v[1] * v[1],
                         0.0,
                         v[3] * v[3] * v[3]};
  double iA[16], iB1[4], iB2[4], iE[16];
  if (!lu_invert(mA, iA, 4, 1e-14) || !lu_invert(mB1, iB1, 2, 1e-14) ||
      !lu_invert(mB2, iB2, 2, 1e-14) || !lu_invert(mE, iE, 4, 1e-14)) {
    err = "a symmetry block of the moment matrix is singular";
    return DBM_ERR_SINGULAR_M;
  }
  for (int k = 0; k < 16; ++k) {
    sp.KA[k] = 0.25 * iA[k];
    sp.KE[k] = ((k / 4) % 2 == 0 ? 0.5 : 0.25) * iE[k];
  }
  for (int k = 0; k < 4; ++k) {
    sp.KB1[k] = 0.25 * iB1[k];
    sp.KB2[k] = 0.25 * iB2[k];
    sp.MB1[k] = mB1[k];
    sp.MB2[k] = mB2[k];
  }
  for (int k = 0; k < 16; ++k) {
    sp.MA[k] = mA[k];
    sp.ME[k] = mE[k];
    sp.iA[k] = iA[k];
    sp.iE[k] = iE[k];
  }
  for (int k = 0; k < 4; ++k) {
    sp.iB1[k] = iB1[k];
    sp.iB2[k] = iB2[k];
  }
  // Self-check: the block projection equals the dense inverse.
  for (int trial = 0; trial < 4; ++trial) {
    double g[kNV], fb[kNV], fd[kNV], scale = 0.0, diff = 0.0;
    for (int k = 0; k < kNV; ++k) g[k] = std::sin(1.3 * k + 0.7 * trial + 0.1) * (1 + k % 3);
    block_project(sp, g, fb);
    for (int r = 0; r < kNV; ++r) {
      double s = 0.0;
      for (int c = 0; c < kNV; ++c) s += sp.Minv[r * kNV + c] * g[c];
      fd[r] = s;
      scale = std::fmax(scale, std::fabs(s));
    }
    for (int r = 0; r < kNV; ++r) diff = std::fmax(diff, std::fabs(fb[r] - fd[r]));
    if (!(diff <= 1e-10 * scale)) {
      err = "symmetry-block projection disagrees with the dense inverse";
      return DBM_ERR_SINGULAR_M;
    }
  }
  // Specular-wall partners: the velocity with one component reversed.
  for (int i = 0; i < kNV; ++i) {
    sp.mirx[i] = sp.miry[i] = -1;
    for (int k = 0; k < kNV; ++k) {
      if (vx[k] == -vx[i] && vy[k] == vy[i] && et[k] == et[i]) sp.mirx[i] = k;
      if (vx[k] == vx[i] && vy[k] == -vy[i] && et[k] == et[i]) sp.miry[i] = k;
    }
    if (sp.mirx[i] < 0 || sp.miry[i] < 0) {
      err = "velocity set is not mirror symmetric";
      return DBM_ERR_ARG;
    }
  }
  // FP32 copies.
  sp.omega_f = (float)sp.omega;
  for (int g = 0; g < 4; ++g) {
    sp.cgx_f[g] = (float)sp.cgx[g];
    sp.cgy_f[g] = (float)sp.cgy[g];
    sp.vg_f[g] = (float)sp.vg[g];
    sp.qg_f[g] = (float)sp.qg[g];
  }
  for (int k = 0; k < 16; ++k) {
    sp.KA_f[k] = (float)sp.KA[k];
    sp.KE_f[k] = (float)sp.KE[k];
    sp.MA_f[k] = (float)sp.MA[k];
    sp.ME_f[k] = (float)sp.ME[k];
  }
  for (int k = 0; k < 4; ++k) {
    sp.KB1_f[k] = (float)sp.KB1[k];
    sp.KB2_f[k] = (float)sp.KB2[k];
    sp.MB1_f[k] = (float)sp.MB1[k];
    sp.MB2_f[k] = (float)sp.MB2[k];
    sp.wB1_f[k] = (float)(sp.omega * iB1[k]);
    sp.wB2_f[k] = (float)(sp.omega * iB2[k]);
  }
  for (int k = 0; k < 16; ++k) sp.wE_f[k] = (float)(sp.omega * iE[k]);
  return DBM_OK;
}

// Reference equilibrium of OM storage for one species and grid row: fref =
// f^eq(n_ref, 0, T_ref) = M^{-1} fhat(n_ref, 0, 0, T_ref/m) (fhat at rest: the
// closed forms listed after Eq.(14) with u = 0), and its A-block moments
// sref: out[0..15] = fref, out[16..19] = sref.
void om_reference(const SpeciesDev &sp, double n_ref, double T_ref, double *out) {
  const double th = T_ref * sp.inv_m, K = sp.K;
  double h[kNV] = {0};
  h[0] = n_ref;
  h[3] = n_ref * K * th;
  h[4] = h[6] = n_ref * th;
  h[13] = h[15] = n_ref * th * (K + 2.0) * th;
  for (int r = 0; r < kNV; ++r) {
    double s = 0.0;
    for (int c = 0; c < kNV; ++c) s += sp.Minv[r * kNV + c] * h[c];
    out[r] = s;
  }
  double *sref = out + kNV;
  for (int j = 0; j < 4; ++j) sref[j] = 0.0;
  for (int i = 0; i < kNV; ++i) {
    const double f = out[i];
    sref[0] += sp.M[0 * kNV + i] * f;
    sref[1] += sp.M[3 * kNV + i] * f;
    sref[2] += (sp.M[4 * kNV + i] + sp.M[6 * kNV + i]) * f;
    sref[3] += (sp.M[13 * kNV + i] + sp.M[15 * kNV + i]) * f;
  }
}

}  // namespace dbm
