// dbm_kernels.hip -- gfx950 kernels of libdbm.
//
// Data layout in HBM (per instance): three distribution buffers, each
// [S][16][ny][nx] in the storage precision (float for FP32-bulk, double for
// FP64), x fastest, so every velocity plane is a dense 2-D array and a
// wavefront's 64 lanes read 64 consecutive cells of one plane per load.
//
// The one-pass stage kernel (k_fused_stage) gives each wavefront a tile of
// 60 output columns (64 lanes with two guard lanes on each side) by `rows`
// rows and marches it in +y:
//   * x-neighbours of the NND stencil come from adjacent lanes through DPP
//     whole-wavefront shifts (no LDS, no barriers);
//   * y-neighbours are carried in registers from row to row (three values per
//     plane with a nonzero v_y, one prefetched value for the others), so each
//     value of f is loaded once per tile plus a four-row halo;
//   * per cell, the moments feeding T are summed in FP64, the mixture u, T,
//     reaction and force terms are evaluated in FP64, and f^eq = M^{-1} fhat
//     is formed through the symmetry blocks of M (56 multiply-adds instead of
//     256) before the BGK + source + Runge-Kutta combine and a single store.
// Tiles are taken from a table in an order that keeps x-neighbouring tiles on
// the same XCD (one L2 per XCD) so that the guard columns hit in L2.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dbm.h"
#include "dbm_internal.hpp"

namespace dbm {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
template <typename T> struct Tab;
template <> struct Tab<float> {
  static __device__ __forceinline__ const float *KA(const SpeciesDev &s) { return s.KA_f; }
  static __device__ __forceinline__ const float *KB1(const SpeciesDev &s) { return s.KB1_f; }
  static __device__ __forceinline__ const float *KB2(const SpeciesDev &s) { return s.KB2_f; }
  static __device__ __forceinline__ const float *KE(const SpeciesDev &s) { return s.KE_f; }
  static __device__ __forceinline__ float cgx(const SpeciesDev &s, int g) { return s.cgx_f[g]; }
  static __device__ __forceinline__ float cgy(const SpeciesDev &s, int g) { return s.cgy_f[g]; }
  static __device__ __forceinline__ float omega(const SpeciesDev &s) { return s.omega_f; }
};
template <> struct Tab<double> {
  static __device__ __forceinline__ const double *KA(const SpeciesDev &s) { return s.KA; }
  static __device__ __forceinline__ const double *KB1(const SpeciesDev &s) { return s.KB1; }
  static __device__ __forceinline__ const double *KB2(const SpeciesDev &s) { return s.KB2; }
  static __device__ __forceinline__ const double *KE(const SpeciesDev &s) { return s.KE; }
  static __device__ __forceinline__ double cgx(const SpeciesDev &s, int g) { return s.cgx[g]; }
  static __device__ __forceinline__ double cgy(const SpeciesDev &s, int g) { return s.cgy[g]; }
  static __device__ __forceinline__ double omega(const SpeciesDev &s) { return s.omega; }
};

// DPP whole-wavefront shifts: shr1 gives lane i the value of lane i-1,
// shl1 the value of lane i+1; the lane with no source keeps `old`.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

__device__ __forceinline__ float dpp_shr1(float src, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                    kDppWaveShr1, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_shl1(float src, float old) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                    kDppWaveShl1, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_shr1(double src, double old) {
  int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), kDppWaveShr1,
                                       0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), kDppWaveShr1,
                                       0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double dpp_shl1(double src, double old) {
  int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), kDppWaveShl1,
                                       0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), kDppWaveShl1,
                                       0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// minmod(a, b) = median(a, b, 0): the smaller-magnitude argument when both
// have the same sign, else 0.
__device__ __forceinline__ float minmod(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Limited slope at a cell for a positive (P) or negative (N) velocity
// component; LIM_NONE gives the unlimited upwind second-order slope.
template <int LIM, typename T> __device__ __forceinline__ T slope_pos(T dlo, T dhi) {
  if constexpr (LIM == DBM_LIM_MINMOD) return minmod(dlo, dhi); else return dlo;
}
template <int LIM, typename T> __device__ __forceinline__ T slope_neg(T dlo, T dhi) {
  if constexpr (LIM == DBM_LIM_MINMOD) return minmod(dlo, dhi); else return dhi;
}

// Velocity signs of plane i (Eq.15 ordering) and its specular partners.
__host__ __device__ constexpr int plane_sx(int i) {
  return ((i >> 2) & 1) == 0 ? ((i & 3) == 0 ? 1 : ((i & 3) == 2 ? -1 : 0))
                             : (((i & 3) == 0 || (i & 3) == 3) ? 1 : -1);
}
__host__ __device__ constexpr int plane_sy(int i) {
  return ((i >> 2) & 1) == 0 ? ((i & 3) == 1 ? 1 : ((i & 3) == 3 ? -1 : 0))
                             : (((i & 3) == 0 || (i & 3) == 1) ? 1 : -1);
}
__host__ __device__ constexpr int mirror_y(int i) {
  return ((i >> 2) & 1) == 0 ? ((i & ~3) | ((i & 3) == 1 ? 3 : ((i & 3) == 3 ? 1 : (i & 3))))
                             : ((i & ~3) | (3 - (i & 3)));
}

__device__ __forceinline__ int map_x(int c, int n, int bc) {
  if (c >= 0 && c < n) return c;
  if (bc == BC_PERIODIC) {
    int r = c % n;
    return r < 0 ? r + n : r;
  }
  return c < 0 ? 0 : n - 1;  // outflow: zero-gradient ghosts
}

// Row map for y: periodic wrap, outflow clamp, or specular reflection about
// the wall face (flip = an odd number of reflections).
__device__ __forceinline__ int map_y(int r, int n, int bc, bool &flip) {
  flip = false;
  if (r >= 0 && r < n) return r;
  if (bc == BC_PERIODIC) {
    int q = r % n;
    return q < 0 ? q + n : q;
  }
  if (bc == BC_OUTFLOW) return r < 0 ? 0 : n - 1;
  for (int it = 0; it < 64 && (r < 0 || r >= n); ++it) {
    r = (r < 0) ? (-1 - r) : (2 * n - 1 - r);
    flip = !flip;
  }
  return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

// Block right-hand side of the equilibrium moments, in the order
// rA[0..3], rB1[4..5], rB2[6..7], rX[8..11], rY[12..15] (see SpeciesDev);
// every entry is a combination of the closed forms listed after Eq.(14).
template <typename U>
__device__ __forceinline__ void eq_rhs(U n, U ux, U uy, U th, U K, U *r) {
  const U ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2;
  const U e2 = (K + U(2)) * th + u2, e4 = (K + U(4)) * th + u2;
  r[0] = n;
  r[1] = n * (K * th + u2);
  r[2] = n * (U(2) * th + u2);
  r[3] = n * (U(2) * th * e2 + u2 * e4);
  const U d = n * (ux2 - uy2);
  r[4] = d;
  r[5] = d * e4;
  const U xy = n * ux * uy;
  r[6] = xy;
  r[7] = xy * e4;
  const U nxu = n * ux, nyu = n * uy;
  r[8] = nxu;
  r[9] = nxu * e2;
  r[10] = nxu * (U(3) * th + ux2);
  r[11] = nxu * (th + uy2);
  r[12] = nyu;
  r[13] = nyu * e2;
  r[14] = nyu * (U(3) * th + uy2);
  r[15] = nyu * (th + ux2);
}

// f^eq of one species from its block right-hand side (plane order of Eq.15).
template <typename T>
__device__ __forceinline__ void block_feq(const SpeciesDev &sp, const T *r, T *f) {
  const T *KA = Tab<T>::KA(sp), *KB1 = Tab<T>::KB1(sp), *KB2 = Tab<T>::KB2(sp),
          *KE = Tab<T>::KE(sp);
  T al[4], xi[4], ps[4], be[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T sa = KA[a * 4] * r[0], sx = KE[a * 4] * r[8], sy = KE[a * 4] * r[12];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      sa = fma(KA[a * 4 + j], r[j], sa);
      sx = fma(KE[a * 4 + j], r[8 + j], sx);
      sy = fma(KE[a * 4 + j], r[12 + j], sy);
    }
    al[a] = sa; xi[a] = sx; ps[a] = sy;
  }
  be[0] = fma(KB1[1], r[5], KB1[0] * r[4]);
  be[2] = fma(KB1[3], r[5], KB1[2] * r[4]);
  be[1] = fma(KB2[1], r[7], KB2[0] * r[6]);
  be[3] = fma(KB2[3], r[7], KB2[2] * r[6]);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const T p = al[g] + be[g], m = al[g] - be[g];
    T *o = f + 4 * g;
    if ((g & 1) == 0) {
      o[0] = p + xi[g]; o[1] = m + ps[g]; o[2] = p - xi[g]; o[3] = m - ps[g];
    } else {
      const T s = xi[g] + ps[g], d = xi[g] - ps[g];
      o[0] = p + s; o[1] = m - d; o[2] = p - s; o[3] = m + d;
    }
  }
}

// FP64 raw moments n, j_x, j_y, E = sum f q of one species from its 16 values.
template <typename T>
__device__ __forceinline__ void species_moments(const SpeciesDev &sp, const T *c, double &n,
                                                double &jx, double &jy, double &E) {
  n = jx = jy = E = 0.0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const double c0 = (double)c[4 * g], c1 = (double)c[4 * g + 1], c2 = (double)c[4 * g + 2],
                 c3 = (double)c[4 * g + 3];
    const double A = (c0 + c2) + (c1 + c3);
    double X, Y;
    if ((g & 1) == 0) {
      X = c0 - c2; Y = c1 - c3;
    } else {
      X = (c0 + c3) - (c1 + c2); Y = (c0 + c1) - (c2 + c3);
    }
    n += A;
    jx = fma(sp.vg[g], X, jx);
    jy = fma(sp.vg[g], Y, jy);
    E = fma(sp.qg[g], A, E);
  }
}

// Per-cell scalar chain in FP64: mixture u, T (conservation statement under
// Eq.6), reaction (Eqs.1-2, 5) and the per-species right-hand side of the
// combined equilibrium f^eq(n*,u,T*) + f^eq(n,u+,T+) - f^eq(n,u^s,T^s).
template <typename T, int S>
__device__ __forceinline__ void cell_rhs(const InstDev &I, const SpeciesDev *sp,
                                         const double *n, const double *jx, const double *jy,
                                         const double *E, T r[S][16]) {
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    rho = fma(sp[s].m, n[s], rho);
    px = fma(sp[s].m, jx[s], px);
    py = fma(sp[s].m, jy[s], py);
    e = fma(sp[s].m, E[s], e);
    kn = fma(sp[s].K, n[s], kn);
  }
  const double ux = px / rho, uy = py / rho;
  const double Tm = (e - rho * (ux * ux + uy * uy)) / kn;
  double nst[S];
  double Tst = Tm;
#pragma unroll
  for (int s = 0; s < S; ++s) nst[s] = n[s];
  if (I.react) {
    double nF = 0.0, nO = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s == I.fuel) nF = fmax(n[s], 0.0);
      if (s == I.oxid) nO = fmax(n[s], 0.0);
    }
    double xi = I.k_ov * nF * nO * exp(-I.EaR / Tm) * sp[0].tau;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (sp[s].a < 0.0) xi = fmin(xi, fmax(n[s], 0.0) / (-sp[s].a));
    double kns = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      nst[s] = fma(sp[s].a, xi, n[s]);
      kns = fma(sp[s].K, nst[s], kns);
    }
    Tst = fma(Tm, kn, I.Q2 * xi) / kns;
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    eq_rhs<T>((T)nst[s], (T)ux, (T)uy, (T)(Tst * sp[s].inv_m), (T)sp[s].K, r[s]);
    if (I.force && n[s] > 1e-300) {
      const double inv_n = 1.0 / n[s];
      const double us = jx[s] * inv_n, vs = jy[s] * inv_n;
      const double Ts = sp[s].m * (E[s] * inv_n - us * us - vs * vs) / sp[s].K;
      const double tau = sp[s].tau;
      double Td = Ts;
      if (I.fmode == DBM_FORCE_T_EXACT)
        Td = Ts - sp[s].m * tau * tau * (I.ax * I.ax + I.ay * I.ay) / sp[s].K;
      double r1[16], r2[16];
      eq_rhs<double>(n[s], us + tau * I.ax, vs + tau * I.ay, Td * sp[s].inv_m, sp[s].K, r1);
      eq_rhs<double>(n[s], us, vs, Ts * sp[s].inv_m, sp[s].K, r2);
#pragma unroll
      for (int k = 0; k < 16; ++k) r[s][k] += (T)(r1[k] - r2[k]);
    }
  }
}

// Bijection of [0, n) that gives XCD x (wavefronts v with v % 8 == x) the
// contiguous chunk x of the tile order.
__device__ __forceinline__ int xcd_remap(int v, int n) {
  const int per = n / kNumXcd, rem = n % kNumXcd;
  const int xcd = v % kNumXcd, local = v / kNumXcd;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// ---------------------------------------------------------------------------
// One-pass stage kernel
// out = alpha * f^n + beta * (f + dt (C(f) + S(f)))   (RKC)
// out = f + dt (C(f) + S(f))                          (!RKC)
// ---------------------------------------------------------------------------
template <typename T, int S, int LIM, bool RKC>
__device__ __forceinline__ void fused_tile(const InstDev &I, int x0, int y0, int rows,
                                           int in_idx, int fn_idx, int out_idx, T alpha,
                                           T beta) {
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = I.nx, ny = I.ny, bcy = I.bcy;
  const SpeciesDev *sp = I.sp;
  const T *__restrict__ fin = (const T *)I.buf[in_idx];
  const T *__restrict__ fnb = (const T *)I.buf[fn_idx];
  T *__restrict__ fout = (T *)I.buf[out_idx];
  const size_t plane = (size_t)nx * (size_t)ny;
  const int col = x0 - 2 + lane;                   // column held by this lane
  const int lcol = map_x(col, nx, I.bcx);          // where its value lives
  const bool writer = lane >= 2 && lane < kWave - 2 && col < nx;

  auto load = [&](int s, int i, int roff, bool flip) -> T {
    const int p = flip ? mirror_y(i) : i;
    return fin[(size_t)(s * kNV + p) * plane + (size_t)(roff + lcol)];
  };

  // State carried between rows.  For plane i of species s:
  //   c  = f at the current row k (all planes)
  //   y1 = f_k - f_{k-1}           (v_y > 0)   or f_{k+1}   (v_y < 0)
  //   y2 = slope at row k-1        (v_y > 0)   or slope at row k (v_y < 0)
  T c[S][kNV], y1[S][kNV], y2[S][kNV];
  {
    bool fm2, fm1, f0, fp1;
    const int rm2 = map_y(y0 - 2, ny, bcy, fm2) * nx, rm1 = map_y(y0 - 1, ny, bcy, fm1) * nx;
    const int r0 = map_y(y0, ny, bcy, f0) * nx, rp1 = map_y(y0 + 1, ny, bcy, fp1) * nx;
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int i = 0; i < kNV; ++i) {
        const int sy = plane_sy(i);
        if (sy > 0) {
          const T a = load(s, i, rm2, fm2), b = load(s, i, rm1, fm1), cc = load(s, i, r0, f0);
          c[s][i] = cc;
          y1[s][i] = cc - b;
          y2[s][i] = slope_pos<LIM>(b - a, cc - b);
        } else if (sy < 0) {
          const T a = load(s, i, rm1, fm1), cc = load(s, i, r0, f0), n1 = load(s, i, rp1, fp1);
          c[s][i] = cc;
          y1[s][i] = n1;
          y2[s][i] = slope_neg<LIM>(cc - a, n1 - cc);
        } else {
          c[s][i] = load(s, i, r0, f0);
          y1[s][i] = T(0);
          y2[s][i] = T(0);
        }
      }
    }
  }

  for (int k = y0; k < y0 + rows; ++k) {
    bool fk1, fk2;
    const int rk1 = map_y(k + 1, ny, bcy, fk1) * nx;
    const int rk2 = map_y(k + 2, ny, bcy, fk2) * nx;
    const int rk = k * nx;

    // Moments and per-cell chain (FP64) from the centre values.
    double n[S], jx[S], jy[S], E[S];
#pragma unroll
    for (int s = 0; s < S; ++s) species_moments<T>(sp[s], c[s], n[s], jx[s], jy[s], E[s]);
    T r[S][16];
    cell_rhs<T, S>(I, sp, n, jx, jy, E, r);

#pragma unroll
    for (int s = 0; s < S; ++s) {
      T feq[kNV];
      block_feq<T>(sp[s], r[s], feq);
      const T om = Tab<T>::omega(sp[s]);
#pragma unroll
      for (int i = 0; i < kNV; ++i) {
        const int g = i >> 2, sx = plane_sx(i), sy = plane_sy(i);
        const T f = c[s][i];
        T acc = f;
        // x: NND difference from adjacent lanes.
        if (sx != 0) {
          const T fm1 = dpp_shr1(f, f), fp1 = dpp_shl1(f, f);
          T Dx;
          if (sx > 0) {
            const T fm2 = dpp_shr1(fm1, fm1);
            const T d0 = f - fm1, dp = fp1 - f, dm = fm1 - fm2;
            Dx = d0 + T(0.5) * (slope_pos<LIM>(d0, dp) - slope_pos<LIM>(dm, d0));
          } else {
            const T fp2 = dpp_shl1(fp1, fp1);
            const T dlo = fp1 - f, dhi = fp2 - fp1, dm = f - fm1;
            Dx = dlo - T(0.5) * (slope_neg<LIM>(dlo, dhi) - slope_neg<LIM>(dm, dlo));
          }
          const T cx = Tab<T>::cgx(sp[s], g);
          acc = (sx > 0) ? fma(-cx, Dx, acc) : fma(cx, Dx, acc);
        }
        // y: NND difference from the carried rows; advance the state.
        if (sy > 0) {
          const T fnew = load(s, i, rk1, fk1);
          const T dn = fnew - f;
          const T sk = slope_pos<LIM>(y1[s][i], dn);
          const T Dy = y1[s][i] + T(0.5) * (sk - y2[s][i]);
          acc = fma(-Tab<T>::cgy(sp[s], g), Dy, acc);
          c[s][i] = fnew;
          y1[s][i] = dn;
          y2[s][i] = sk;
        } else if (sy < 0) {
          const T fnew = load(s, i, rk2, fk2);
          const T n1 = y1[s][i];
          const T dlo = n1 - f, dhi = fnew - n1;
          const T tk1 = slope_neg<LIM>(dlo, dhi);
          const T Dy = dlo - T(0.5) * (tk1 - y2[s][i]);
          acc = fma(Tab<T>::cgy(sp[s], g), Dy, acc);
          c[s][i] = n1;
          y1[s][i] = fnew;
          y2[s][i] = tk1;
        } else {
          c[s][i] = load(s, i, rk1, fk1);
        }
        T res = fma(om, feq[i] - f, acc);
        const size_t o = (size_t)(s * kNV + i) * plane + (size_t)(rk + col);
        if constexpr (RKC) {
          const T fnv = fnb[(size_t)(s * kNV + i) * plane + (size_t)(rk + lcol)];
          res = fma(alpha, fnv, beta * res);
        }
        if (writer) fout[o] = res;
      }
    }
  }
}

template <typename T, int S, int LIM, bool RKC>
__global__ __launch_bounds__(kWave) void k_fused_stage(const InstDev *__restrict__ insts,
                                                       const Tile *__restrict__ tiles,
                                                       int ntiles, int in_idx, int fn_idx,
                                                       int out_idx, T alpha, T beta) {
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile t = tiles[xcd_remap(v, ntiles)];
    fused_tile<T, S, LIM, RKC>(insts[t.inst], t.x0, t.y0, t.rows, in_idx, fn_idx, out_idx,
                               alpha, beta);
  }
}

// ---------------------------------------------------------------------------
// Plain path: one thread per cell for the equilibrium (dense FP64 M^{-1}),
// one thread per (cell, plane) for convection + combine.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void plain_feq_cell(const InstDev &I, const T *f, size_t plane,
                                               size_t cell, T *dst) {
  const int S = I.S;
  const SpeciesDev *sp = I.sp;
  double n[kMaxSpecies], jx[kMaxSpecies], jy[kMaxSpecies], E[kMaxSpecies];
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
  for (int s = 0; s < S; ++s) {
    double a = 0, b = 0, cc = 0, d = 0;
    for (int i = 0; i < kNV; ++i) {
      const double v = (double)f[(size_t)(s * kNV + i) * plane + cell];
      const double vx = sp[s].M[1 * kNV + i], vy = sp[s].M[2 * kNV + i], q = sp[s].M[3 * kNV + i];
      a += v;
      b = fma(v, vx, b);
      cc = fma(v, vy, cc);
      d = fma(v, q, d);
    }
    n[s] = a; jx[s] = b; jy[s] = cc; E[s] = d;
    rho = fma(sp[s].m, a, rho);
    px = fma(sp[s].m, b, px);
    py = fma(sp[s].m, cc, py);
    e = fma(sp[s].m, d, e);
    kn = fma(sp[s].K, a, kn);
  }
  const double ux = px / rho, uy = py / rho;
  const double Tm = (e - rho * (ux * ux + uy * uy)) / kn;
  double Tst = Tm, xi = 0.0;
  if (I.react) {
    const double nF = fmax(n[I.fuel], 0.0), nO = fmax(n[I.oxid], 0.0);
    xi = I.k_ov * nF * nO * exp(-I.EaR / Tm) * sp[0].tau;
    for (int s = 0; s < S; ++s)
      if (sp[s].a < 0.0) xi = fmin(xi, fmax(n[s], 0.0) / (-sp[s].a));
    double kns = 0.0;
    for (int s = 0; s < S; ++s) kns = fma(sp[s].K, fma(sp[s].a, xi, n[s]), kns);
    Tst = fma(Tm, kn, I.Q2 * xi) / kns;
  }
  for (int s = 0; s < S; ++s) {
    // the sixteen closed forms listed after Eq.(14)
    auto fhat = [&](double nn, double u, double v, double th, double *h) {
      const double K = sp[s].K, u2 = u * u + v * v;
      const double e2 = (K + 2.0) * th + u2, e4 = (K + 4.0) * th + u2;
      h[0] = nn; h[1] = nn * u; h[2] = nn * v; h[3] = nn * (K * th + u2);
      h[4] = nn * (th + u * u); h[5] = nn * u * v; h[6] = nn * (th + v * v);
      h[7] = nn * u * e2; h[8] = nn * v * e2;
      h[9] = nn * u * (3.0 * th + u * u); h[10] = nn * v * (th + u * u);
      h[11] = nn * u * (th + v * v); h[12] = nn * v * (3.0 * th + v * v);
      h[13] = nn * (th * e2 + u * u * e4); h[14] = nn * u * v * e4;
      h[15] = nn * (th * e2 + v * v * e4);
    };
    double g[kNV], h1[kNV], h2[kNV];
    fhat(fma(sp[s].a, xi, n[s]), ux, uy, Tst * sp[s].inv_m, g);
    if (I.force && n[s] > 1e-300) {
      const double us = jx[s] / n[s], vs = jy[s] / n[s];
      const double Ts = sp[s].m * (E[s] / n[s] - us * us - vs * vs) / sp[s].K;
      const double tau = sp[s].tau;
      const double Td = (I.fmode == DBM_FORCE_T_EXACT)
                            ? Ts - sp[s].m * tau * tau * (I.ax * I.ax + I.ay * I.ay) / sp[s].K
                            : Ts;
      fhat(n[s], us + tau * I.ax, vs + tau * I.ay, Td * sp[s].inv_m, h1);
      fhat(n[s], us, vs, Ts * sp[s].inv_m, h2);
      for (int k = 0; k < kNV; ++k) g[k] += h1[k] - h2[k];
    }
    for (int r = 0; r < kNV; ++r) {
      double acc = 0.0;
      for (int k = 0; k < kNV; ++k) acc = fma(sp[s].Minv[r * kNV + k], g[k], acc);
      dst[(size_t)(s * kNV + r) * plane + cell] = (T)acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_plain_eq(const InstDev *__restrict__ insts, int inst,
                                                  int in_idx) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  plain_feq_cell<T>(I, (const T *)I.buf[in_idx], plane, cell, (T *)I.scratch);
}

// Map a possibly-ghost index along one axis; walls reflect and flip.
__device__ __forceinline__ int map_axis(int j, int n, int bc, int &flips) {
  if (j >= 0 && j < n) return j;
  if (bc == BC_PERIODIC) {
    int q = j % n;
    return q < 0 ? q + n : q;
  }
  if (bc == BC_OUTFLOW) return j < 0 ? 0 : n - 1;
  for (int it = 0; it < 64 && (j < 0 || j >= n); ++it) {
    j = (j < 0) ? (-1 - j) : (2 * n - 1 - j);
    flips ^= 1;
  }
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

template <typename T>
__device__ __forceinline__ T plain_value(const InstDev &I, const T *f, size_t plane, int s,
                                         int i, int x, int y) {
  int fx = 0, fy = 0;
  const int mx = map_axis(x, I.nx, I.bcx, fx), my = map_axis(y, I.ny, I.bcy, fy);
  int p = i;
  if (fx) p = I.sp[s].mirx[p];
  if (fy) p = I.sp[s].miry[p];
  return f[(size_t)(s * kNV + p) * plane + (size_t)my * I.nx + mx];
}

template <typename T>
__device__ __forceinline__ T nnd_face(T fm1, T f0, T fp1, T fp2, int sgn, int lim) {
  if (sgn > 0) {
    const T sl = lim == DBM_LIM_MINMOD ? minmod(f0 - fm1, fp1 - f0) : (f0 - fm1);
    return f0 + T(0.5) * sl;
  }
  const T sl = lim == DBM_LIM_MINMOD ? minmod(fp1 - f0, fp2 - fp1) : (fp2 - fp1);
  return fp1 - T(0.5) * sl;
}

template <typename T>
__global__ __launch_bounds__(256) void k_plain_update(const InstDev *__restrict__ insts,
                                                      int inst, int in_idx, int fn_idx,
                                                      int out_idx, T alpha, T beta, int rkc) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const int si = blockIdx.y, s = si / kNV, i = si % kNV;
  const int x = (int)(cell % I.nx), y = (int)(cell / I.nx);
  const T *f = (const T *)I.buf[in_idx];
  const SpeciesDev &sp = I.sp[s];
  const double vx = sp.M[1 * kNV + i], vy = sp.M[2 * kNV + i];
  const T fc = f[(size_t)si * plane + cell];
  T C = T(0);
  if (vx != 0.0) {
    T w[5];
    for (int k = 0; k < 5; ++k) w[k] = plain_value<T>(I, f, plane, s, i, x - 2 + k, y);
    const int sg = vx > 0 ? 1 : -1;
    const T fr = nnd_face<T>(w[1], w[2], w[3], w[4], sg, I.lim);
    const T fl = nnd_face<T>(w[0], w[1], w[2], w[3], sg, I.lim);
    C -= (T)(vx * I.dt / I.dx) * (fr - fl);
  }
  if (vy != 0.0) {
    T w[5];
    for (int k = 0; k < 5; ++k) w[k] = plain_value<T>(I, f, plane, s, i, x, y - 2 + k);
    const int sg = vy > 0 ? 1 : -1;
    const T fr = nnd_face<T>(w[1], w[2], w[3], w[4], sg, I.lim);
    const T fl = nnd_face<T>(w[0], w[1], w[2], w[3], sg, I.lim);
    C -= (T)(vy * I.dt / I.dy) * (fr - fl);
  }
  const T feq = ((const T *)I.scratch)[(size_t)si * plane + cell];
  T res = fc + C + (T)sp.omega * (feq - fc);
  if (rkc) res = alpha * ((const T *)I.buf[fn_idx])[(size_t)si * plane + cell] + beta * res;
  ((T *)I.buf[out_idx])[(size_t)si * plane + cell] = res;
}

// ---------------------------------------------------------------------------
// Initialisation, diagnostics, conversion
// ---------------------------------------------------------------------------
// f := f^eq(n^s, u, T); fields = [n_sp (S planes), ux, uy, T] in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_init_eq(const InstDev *__restrict__ insts, int inst,
                                                 const double *__restrict__ fields,
                                                 int out_idx) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const int S = I.S;
  const double ux = fields[(size_t)S * plane + cell], uy = fields[(size_t)(S + 1) * plane + cell];
  const double Tm = fields[(size_t)(S + 2) * plane + cell];
  T *out = (T *)I.buf[out_idx];
  for (int s = 0; s < S; ++s) {
    const SpeciesDev &sp = I.sp[s];
    const double nn = fields[(size_t)s * plane + cell], th = Tm * sp.inv_m, K = sp.K;
    const double u2 = ux * ux + uy * uy;
    const double e2 = (K + 2.0) * th + u2, e4 = (K + 4.0) * th + u2;
    const double h[kNV] = {nn,
                           nn * ux,
                           nn * uy,
                           nn * (K * th + u2),
                           nn * (th + ux * ux),
                           nn * ux * uy,
                           nn * (th + uy * uy),
                           nn * ux * e2,
                           nn * uy * e2,
                           nn * ux * (3.0 * th + ux * ux),
                           nn * uy * (th + ux * ux),
                           nn * ux * (th + uy * uy),
                           nn * uy * (3.0 * th + uy * uy),
                           nn * (th * e2 + ux * ux * e4),
                           nn * ux * uy * e4,
                           nn * (th * e2 + uy * uy * e4)};
    for (int r = 0; r < kNV; ++r) {
      double acc = 0.0;
      for (int k = 0; k < kNV; ++k) acc = fma(sp.Minv[r * kNV + k], h[k], acc);
      out[(size_t)(s * kNV + r) * plane + cell] = (T)acc;
    }
  }
}

// Per-cell species moments in FP64 (dense rows of M).
template <typename T>
__device__ __forceinline__ void dense_moments(const InstDev &I, const T *f, size_t plane,
                                              size_t cell, int s, double &n, double &jx,
                                              double &jy, double &E) {
  const SpeciesDev &sp = I.sp[s];
  n = jx = jy = E = 0.0;
  for (int i = 0; i < kNV; ++i) {
    const double v = (double)f[(size_t)(s * kNV + i) * plane + cell];
    n += v;
    jx = fma(v, sp.M[1 * kNV + i], jx);
    jy = fma(v, sp.M[2 * kNV + i], jy);
    E = fma(v, sp.M[3 * kNV + i], E);
  }
}

// dst = [rho_sp (S planes), ux, uy, T]
template <typename T>
__global__ __launch_bounds__(256) void k_moments(const InstDev *__restrict__ insts, int inst,
                                                 int in_idx, double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const T *f = (const T *)I.buf[in_idx];
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
  for (int s = 0; s < I.S; ++s) {
    double n, jx, jy, E;
    dense_moments<T>(I, f, plane, cell, s, n, jx, jy, E);
    const double m = I.sp[s].m;
    dst[(size_t)s * plane + cell] = m * n;
    rho = fma(m, n, rho);
    px = fma(m, jx, px);
    py = fma(m, jy, py);
    e = fma(m, E, e);
    kn = fma(I.sp[s].K, n, kn);
  }
  const double ux = px / rho, uy = py / rho;
  dst[(size_t)I.S * plane + cell] = ux;
  dst[(size_t)(I.S + 1) * plane + cell] = uy;
  dst[(size_t)(I.S + 2) * plane + cell] = (e - rho * (ux * ux + uy * uy)) / kn;
}

// Eqs.(17)-(20) for species `which`: dst = [12][cells].
template <typename T>
__global__ __launch_bounds__(256) void k_noneq(const InstDev *__restrict__ insts, int inst,
                                               int in_idx, int which,
                                               double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const T *f = (const T *)I.buf[in_idx];
  double rho = 0, px = 0, py = 0, e = 0, kn = 0, nw = 0;
  for (int s = 0; s < I.S; ++s) {
    double n, jx, jy, E;
    dense_moments<T>(I, f, plane, cell, s, n, jx, jy, E);
    const double m = I.sp[s].m;
    if (s == which) nw = n;
    rho = fma(m, n, rho);
    px = fma(m, jx, px);
    py = fma(m, jy, py);
    e = fma(m, E, e);
    kn = fma(I.sp[s].K, n, kn);
  }
  const double ux = px / rho, uy = py / rho;
  const double Tm = (e - rho * (ux * ux + uy * uy)) / kn;
  const SpeciesDev &sp = I.sp[which];
  const double th = Tm * sp.inv_m, K = sp.K, u2 = ux * ux + uy * uy;
  const double e2 = (K + 2.0) * th + u2, e4 = (K + 4.0) * th + u2;
  const double h[kNV] = {nw,
                         nw * ux,
                         nw * uy,
                         nw * (K * th + u2),
                         nw * (th + ux * ux),
                         nw * ux * uy,
                         nw * (th + uy * uy),
                         nw * ux * e2,
                         nw * uy * e2,
                         nw * ux * (3.0 * th + ux * ux),
                         nw * uy * (th + ux * ux),
                         nw * ux * (th + uy * uy),
                         nw * uy * (3.0 * th + uy * uy),
                         nw * (th * e2 + ux * ux * e4),
                         nw * ux * uy * e4,
                         nw * (th * e2 + uy * uy * e4)};
  double dfv[kNV];
  for (int r = 0; r < kNV; ++r) {
    double acc = 0.0;
    for (int k = 0; k < kNV; ++k) acc = fma(sp.Minv[r * kNV + k], h[k], acc);
    dfv[r] = (double)f[(size_t)(which * kNV + r) * plane + cell] - acc;
  }
  for (int row = 4; row < kNV; ++row) {
    double acc = 0.0;
    for (int i = 0; i < kNV; ++i) acc = fma(sp.M[row * kNV + i], dfv[i], acc);
    dst[(size_t)(row - 4) * plane + cell] = sp.m * acc;
  }
}

// Wavefront sum by DPP-free cross-lane shuffles (FP64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

constexpr int kTotBlocks = 512;
constexpr int kTotThreads = 256;

// Partial totals per block: [block][S+3] = mass^s, Px, Py, E (unscaled).
template <typename T>
__global__ __launch_bounds__(kTotThreads) void k_totals_partial(const InstDev *__restrict__ insts,
                                                                int inst, int in_idx,
                                                                double *__restrict__ part) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const T *f = (const T *)I.buf[in_idx];
  const int S = I.S, nq = S + 3;
  double acc[kMaxSpecies + 3];
  for (int q = 0; q < nq; ++q) acc[q] = 0.0;
  for (size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cell < plane;
       cell += (size_t)gridDim.x * blockDim.x) {
    for (int s = 0; s < S; ++s) {
      double n, jx, jy, E;
      dense_moments<T>(I, f, plane, cell, s, n, jx, jy, E);
      const double m = I.sp[s].m;
      acc[s] = fma(m, n, acc[s]);
      acc[S] = fma(m, jx, acc[S]);
      acc[S + 1] = fma(m, jy, acc[S + 1]);
      acc[S + 2] = fma(0.5 * m, E, acc[S + 2]);
    }
  }
  __shared__ double red[kTotThreads / kWave][kMaxSpecies + 3];
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  for (int q = 0; q < nq; ++q) {
    const double v = wave_sum(acc[q]);
    if (l == 0) red[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    double s = 0.0;
    for (int k = 0; k < kTotThreads / kWave; ++k) s += red[k][threadIdx.x];
    part[(size_t)blockIdx.x * nq + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(64) void k_totals_final(const double *__restrict__ part, int nblocks,
                                                     int nq, double area,
                                                     double *__restrict__ out) {
  const int q = threadIdx.x;
  if (q >= nq) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * nq + q];
  out[q] = s * area;
}

template <typename T>
__global__ __launch_bounds__(256) void k_widen(const T *__restrict__ src, double *__restrict__ dst,
                                               size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (double)src[k];
}
template <typename T>
__global__ __launch_bounds__(256) void k_narrow(const double *__restrict__ src, T *__restrict__ dst,
                                                size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (T)src[k];
}

// Non-finite values, or a species density below -1e-12 of the local total.
template <typename T>
__global__ __launch_bounds__(256) void k_check(const InstDev *__restrict__ insts, int inst,
                                               int in_idx, int *__restrict__ flag) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const T *f = (const T *)I.buf[in_idx];
  double tot = 0.0, nmin = 0.0;
  bool bad = false;
  for (int s = 0; s < I.S; ++s) {
    double n = 0.0;
    for (int i = 0; i < kNV; ++i) {
      const double v = (double)f[(size_t)(s * kNV + i) * plane + cell];
      bad |= !isfinite(v);
      n += v;
    }
    tot += n;
    nmin = fmin(nmin, n);
  }
  if (bad || nmin < -1e-12 * fabs(tot)) atomicOr(flag, 1);
}

// Lane-layout probe of the DPP shifts used above: out[l] = shr1(l),
// out[64+l] = shl1(l), with old = -1.
__global__ __launch_bounds__(64) void k_dpp_probe(int *__restrict__ out) {
  const int l = threadIdx.x;
  const float v = (float)l;
  out[l] = (int)dpp_shr1(v, -1.0f);
  out[64 + l] = (int)dpp_shl1(v, -1.0f);
  const double d = (double)l;
  out[128 + l] = (int)dpp_shr1(d, -1.0);
  out[192 + l] = (int)dpp_shl1(d, -1.0);
}

// A single wavefront that idles for `ticks` of the constant-rate wall clock
// (bounded by an iteration cap), used to let the host queue timed launches.
__global__ __launch_bounds__(64) void k_delay(unsigned long long ticks) {
  const unsigned long long t0 = wall_clock64();
  for (int it = 0; it < (1 << 24); ++it) {
    if (wall_clock64() - t0 >= ticks) break;
    __builtin_amdgcn_s_sleep(4);
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from dbm_api.cpp)
// ---------------------------------------------------------------------------
template <typename T, int S, int LIM, bool RKC>
static hipError_t launch_fused_t(const InstDev *insts, const Tile *tiles, int ntiles, int grid,
                                 int in_idx, int fn_idx, int out_idx, double alpha, double beta,
                                 hipStream_t st) {
  hipLaunchKernelGGL((k_fused_stage<T, S, LIM, RKC>), dim3(grid), dim3(kWave), 0, st, insts,
                     tiles, ntiles, in_idx, fn_idx, out_idx, (T)alpha, (T)beta);
  return hipGetLastError();
}

template <typename T, int S, int LIM>
static hipError_t launch_fused_s(bool rkc, const InstDev *insts, const Tile *tiles, int ntiles,
                                 int grid, int a, int b, int c, double al, double be,
                                 hipStream_t st) {
  return rkc ? launch_fused_t<T, S, LIM, true>(insts, tiles, ntiles, grid, a, b, c, al, be, st)
             : launch_fused_t<T, S, LIM, false>(insts, tiles, ntiles, grid, a, b, c, al, be, st);
}

template <typename T, int S>
static hipError_t launch_fused_l(int lim, bool rkc, const InstDev *insts, const Tile *tiles,
                                 int ntiles, int grid, int a, int b, int c, double al, double be,
                                 hipStream_t st) {
  return lim == DBM_LIM_MINMOD
             ? launch_fused_s<T, S, DBM_LIM_MINMOD>(rkc, insts, tiles, ntiles, grid, a, b, c, al,
                                                    be, st)
             : launch_fused_s<T, S, DBM_LIM_NONE>(rkc, insts, tiles, ntiles, grid, a, b, c, al,
                                                  be, st);
}

template <typename T>
static hipError_t launch_fused_p(int S, int lim, bool rkc, const InstDev *insts,
                                 const Tile *tiles, int ntiles, int grid, int a, int b, int c,
                                 double al, double be, hipStream_t st) {
  switch (S) {
    case 1: return launch_fused_l<T, 1>(lim, rkc, insts, tiles, ntiles, grid, a, b, c, al, be, st);
    case 2: return launch_fused_l<T, 2>(lim, rkc, insts, tiles, ntiles, grid, a, b, c, al, be, st);
    case 3: return launch_fused_l<T, 3>(lim, rkc, insts, tiles, ntiles, grid, a, b, c, al, be, st);
    case 4: return launch_fused_l<T, 4>(lim, rkc, insts, tiles, ntiles, grid, a, b, c, al, be, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused(bool fp32, int S, int lim, bool rkc, const InstDev *insts,
                        const Tile *tiles, int ntiles, int grid, int in_idx, int fn_idx,
                        int out_idx, double alpha, double beta, hipStream_t st) {
  return fp32 ? launch_fused_p<float>(S, lim, rkc, insts, tiles, ntiles, grid, in_idx, fn_idx,
                                      out_idx, alpha, beta, st)
              : launch_fused_p<double>(S, lim, rkc, insts, tiles, ntiles, grid, in_idx, fn_idx,
                                       out_idx, alpha, beta, st);
}

hipError_t fused_occupancy(bool fp32, int S, int lim, bool rkc, int *waves_per_cu) {
  const void *fn = nullptr;
#define DBM_PICK(T, SS)                                                                         \
  fn = lim == DBM_LIM_MINMOD                                                                   \
           ? (rkc ? (const void *)k_fused_stage<T, SS, DBM_LIM_MINMOD, true>                   \
                  : (const void *)k_fused_stage<T, SS, DBM_LIM_MINMOD, false>)                 \
           : (rkc ? (const void *)k_fused_stage<T, SS, DBM_LIM_NONE, true>                     \
                  : (const void *)k_fused_stage<T, SS, DBM_LIM_NONE, false>)
  if (fp32) {
    switch (S) { case 1: DBM_PICK(float, 1); break; case 2: DBM_PICK(float, 2); break;
                 case 3: DBM_PICK(float, 3); break; case 4: DBM_PICK(float, 4); break;
                 default: return hipErrorInvalidValue; }
  } else {
    switch (S) { case 1: DBM_PICK(double, 1); break; case 2: DBM_PICK(double, 2); break;
                 case 3: DBM_PICK(double, 3); break; case 4: DBM_PICK(double, 4); break;
                 default: return hipErrorInvalidValue; }
  }
#undef DBM_PICK
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(waves_per_cu, fn, kWave, 0);
}

static inline unsigned blocks_for(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_plain(bool fp32, const InstDev *insts, int inst, size_t cells, int S,
                        int in_idx, int fn_idx, int out_idx, double alpha, double beta, bool rkc,
                        hipStream_t st) {
  const dim3 g1(blocks_for(cells, 256)), g2(blocks_for(cells, 256), (unsigned)(S * kNV));
  if (fp32) {
    hipLaunchKernelGGL(k_plain_eq<float>, g1, dim3(256), 0, st, insts, inst, in_idx);
    hipLaunchKernelGGL(k_plain_update<float>, g2, dim3(256), 0, st, insts, inst, in_idx, fn_idx,
                       out_idx, (float)alpha, (float)beta, (int)rkc);
  } else {
    hipLaunchKernelGGL(k_plain_eq<double>, g1, dim3(256), 0, st, insts, inst, in_idx);
    hipLaunchKernelGGL(k_plain_update<double>, g2, dim3(256), 0, st, insts, inst, in_idx,
                       fn_idx, out_idx, alpha, beta, (int)rkc);
  }
  return hipGetLastError();
}

hipError_t launch_init(bool fp32, const InstDev *insts, int inst, size_t cells,
                       const double *fields, int out_idx, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_init_eq<float>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, fields, out_idx);
  else
    hipLaunchKernelGGL(k_init_eq<double>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, fields, out_idx);
  return hipGetLastError();
}

hipError_t launch_moments(bool fp32, const InstDev *insts, int inst, size_t cells, int in_idx,
                          double *dst, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_moments<float>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, dst);
  else
    hipLaunchKernelGGL(k_moments<double>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, dst);
  return hipGetLastError();
}

hipError_t launch_noneq(bool fp32, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int which, double *dst, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_noneq<float>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, which, dst);
  else
    hipLaunchKernelGGL(k_noneq<double>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, which, dst);
  return hipGetLastError();
}

int totals_blocks() { return kTotBlocks; }

hipError_t launch_totals(bool fp32, const InstDev *insts, int inst, int in_idx, int nq,
                         double area, double *partials, double *out, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_totals_partial<float>, dim3(kTotBlocks), dim3(kTotThreads), 0, st,
                       insts, inst, in_idx, partials);
  else
    hipLaunchKernelGGL(k_totals_partial<double>, dim3(kTotBlocks), dim3(kTotThreads), 0, st,
                       insts, inst, in_idx, partials);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partials, kTotBlocks, nq, area,
                     out);
  return hipGetLastError();
}

hipError_t launch_widen(bool fp32, const void *src, double *dst, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_widen<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const float *)src, dst, n);
  else
    hipLaunchKernelGGL(k_widen<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                       (const double *)src, dst, n);
  return hipGetLastError();
}

hipError_t launch_narrow(bool fp32, const double *src, void *dst, size_t n, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_narrow<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, src,
                       (float *)dst, n);
  else
    hipLaunchKernelGGL(k_narrow<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, src,
                       (double *)dst, n);
  return hipGetLastError();
}

hipError_t launch_check(bool fp32, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int *flag, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_check<float>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, flag);
  else
    hipLaunchKernelGGL(k_check<double>, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, flag);
  return hipGetLastError();
}

hipError_t launch_delay(double microseconds, hipStream_t st) {
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  const unsigned long long ticks = (unsigned long long)(microseconds * 1e-3 * (double)khz);
  hipLaunchKernelGGL(k_delay, dim3(1), dim3(64), 0, st, ticks);
  return hipGetLastError();
}

hipError_t launch_dpp_probe(int *out, hipStream_t st) {
  hipLaunchKernelGGL(k_dpp_probe, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

}  // namespace dbm
