// dbm_internal.hpp -- structures shared by the host runtime and the gfx950
// kernels of libdbm.  Everything here lives in the caller's device workspace.
#pragma once

#include <cstddef>
#include <cstdint>

namespace dbm {

constexpr int kNV = 16;        // discrete velocities per species (D2V16)
constexpr int kMaxSpecies = 16;
constexpr int kMaxReact = 4;          // steps of a multi-step mechanism
constexpr int kMaxFusedSpecies = 4;   // one-pass kernels are instantiated for S <= 4
constexpr int kWave = 64;
constexpr int kNumXcd = 8;     // MI355X: 8 accelerator complex dies, one L2 each

enum Bc { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_WALL = 2 };

// Per-species tables of one instance.
//
// The 16 planes form four orbits of four velocities under the symmetry group
// of the square (Eq.15).  Within an orbit g the distribution is rewritten as
//   A_g = sum of the four values, B_g = alternating sum, X_g, Y_g = first
//   moments with the sign of v_x, v_y,
// and the moment matrix M splits into independent blocks acting on
//   (A_a, A_b, A_c, A_d)   rows 1, v^2+eta^2, v_x^2+v_y^2, (v^2+eta^2)(v_x^2+v_y^2)
//   (B_a, B_c)             rows v_x^2-v_y^2, (v^2+eta^2)(v_x^2-v_y^2)
//   (B_b, B_d)             rows v_x v_y, (v^2+eta^2) v_x v_y
//   (X_a, X_b, X_c, X_d)   rows v_x, (v^2+eta^2) v_x, v_x^3, v_x v_y^2
//   (Y_a, Y_b, Y_c, Y_d)   the same block with x and y exchanged.
// MA, MB1, MB2, ME are those blocks (row-major, unknowns in the order above);
// KA, KB1, KB2, KE are their FP64 inverses with the orbit reconstruction
// factors (1/4 for A and B, 1/2 or 1/4 for X and Y) folded in.
struct SpeciesDev {
  // FP64 per-cell scalar chain
  double m, K, tau, a, inv_m;
  double inv_neg_a;      // 1 / (-a) for reactants (a < 0), else 0
  double inv_K;          // 1 / (D + I)
  double vg[4];          // group speed parameter v_g
  double qg[4];          // |v|^2 + eta^2 of group g
  double omega;          // dt / tau
  double cgx[4], cgy[4]; // dt v_g / dx, dt v_g / dy
  double KA[16], KB1[4], KB2[4], KE[16];
  double MA[16], MB1[4], MB2[4], ME[16];  // the blocks themselves (moments of f)
  double Minv[kNV * kNV];  // dense FP64 inverse (plain path, init, diagnostics)
  double M[kNV * kNV];     // dense moment matrix (diagnostics)
  // FP32 copies for the FP32-bulk kernels
  float omega_f;
  float cgx_f[4], cgy_f[4];
  float KA_f[16], KB1_f[4], KB2_f[4], KE_f[16];
  float MA_f[16], MB1_f[4], MB2_f[4], ME_f[16];
  float vg_f[4], qg_f[4];
  int mirx[kNV], miry[kNV];
  // Shifted orbit-moment storage of FP32-bulk f (OM storage).  Per cell and
  // species the 16 stored values are
  //   s[0..3]   the A-block moments (rows 1, v^2+eta^2, v_x^2+v_y^2,
  //             (v^2+eta^2)(v_x^2+v_y^2)) of f - fref: n - n_ref, E - E_ref, ...
  //   s[4..7]   B_a, B_b, B_c, B_d   (orbit alternating sums of f)
  //   s[8..11]  X_a .. X_d           (orbit sums signed by v_x)
  //   s[12..15] Y_a .. Y_d           (orbit sums signed by v_y)
  // with fref = f^eq(n_ref, 0, T_ref) an equilibrium at rest, whose B, X and Y
  // vanish, fixed per grid row (InstDev::rref).  iA, iB1, iB2, iE are the
  // plain inverses of the blocks (moments -> orbit components); the FP32
  // copies of iB and iE carry the factor omega = dt/tau of the collision.
  double iA[16], iB1[4], iB2[4], iE[16];
  float wB1_f[4], wB2_f[4], wE_f[16];
  double sref[4];        // the A-block moments of fref when one reference serves the grid
};

// Elements from one plane of an f buffer to the next: the nx*ny cells plus
// 17 x 256 bytes.  With power-of-two plane sizes the 16 planes of a cell
// otherwise start at one offset of the memory interleave; the stage kernel,
// which reads and writes 16 plane streams per species, measured ~9% slower
// at 4096^2 and 1024^2 without the pad.  `elem_bytes` is 8 (FP64) or 4 (FP32
// and the FP32 part of FP32X, whose bf16 part uses the same element index).
constexpr size_t kPlanePadBytes = 17 * 256;
inline size_t plane_stride(size_t cells, size_t elem_bytes) {
  return cells + kPlanePadBytes / elem_bytes;
}

struct InstDev {
  void *buf[3];          // three f buffers [S][16][ps] (ps >= ny*nx, row-major
                         // [ny][nx] in each plane) in storage precision
  size_t ps;             // plane stride of the f buffers, in elements
  void *scratch;         // per-instance scratch (plain-path f^eq, staging)
  const SpeciesDev *sp;  // S entries
  int nx, ny, bcx, bcy;
  int S;
  // Chemistry: nreact steps of Eq.(2) (0 = none); the one-step reaction is
  // step 0 with the species' stoichiometric coefficients.
  int nreact;
  int rfuel[kMaxReact], roxid[kMaxReact];
  double rk[kMaxReact], rEa[kMaxReact], rQ2[kMaxReact];  // rQ2 = 2 Q_r
  double rdK[kMaxReact];                   // sum_s (D + I^s) a_r^s
  double ra[kMaxReact][kMaxSpecies];       // a_r^s
  double rneg[kMaxReact][kMaxSpecies];     // max(-a_r^s, 0): consumption per extent
  int force, fmode;
  double ax, ay;
  double dt, dx, dy;
  int lim;
  int om;                // FP32-bulk buffers hold OM storage (see SpeciesDev)
  int ares;              // ... with A-block residuals: four uint16 planes per
                         // species (bfloat16 remainders of the A-block values)
                         // after the S x 16 FP32 planes of every buffer
  // OM storage references, one per species and grid row (set with the
  // fields): rref[(s * ny + y) * kRowRef + 0..15] = fref of row y (FP64),
  // + 16..19 = its A-block moments sref; dref[(s * (ny + 4) + y + 2) * 4 +
  // g] = fref(row y+1) - fref(row y) of the planes of velocity group g (equal
  // at rest) rounded once to FP32, for y = -2 .. ny+1 with the rows outside
  // the grid mapped as the y boundary maps them (the stencil's differences
  // between rows add it).
  const double *rref;
  const float *dref;
  // The same per species and grid row y as one record of kRowRec 32-bit
  // words for the one-pass kernel: the group differences of rows y and y+1
  // (words 0..3, 4..7), sref of row y (FP64, words 8..15) and the first two
  // sref of row y+2 (words 16..19; zero past the grid).
  const uint32_t *orec;
};
constexpr int kRowRef = kNV + 4;
constexpr int kRowRec = 20;

// One tile: a wavefront marches `rows` rows of 64 columns starting at (x0, y0).
struct Tile {
  int inst, x0, y0, rows;
};

}  // namespace dbm
