// dbm_api.cpp -- C ABI of libdbm: validation, workspace layout, tile tables,
// the autotuner, HIP graph capture and replay, and the host sides of the
// diagnostics.  See include/dbm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dbm.h"
#include "dbm_internal.hpp"

namespace dbm {
int build_species(const dbm_species &in, const dbm_config &cfg, SpeciesDev &sp, std::string &err);
void om_reference(const SpeciesDev &sp, double n_ref, double T_ref, double *out);
hipError_t launch_fused(int prec, int S, int lim, bool rkc, bool split, bool pipe, bool sr,
                        bool cw, int om, bool ares, bool drain, uint32_t *ctr,
                        const InstDev *insts, const Tile *tiles, int ntiles, int grid,
                        int in_idx, int fn_idx, int out_idx, double alpha, double beta,
                        hipStream_t st);
hipError_t fused_occupancy(int prec, int S, int lim, bool rkc, bool split, bool cw, bool om,
                           bool ares, int *waves_per_cu);
hipError_t launch_plain(int prec, const InstDev *insts, int inst, size_t cells, int S,
                        int in_idx, int fn_idx, int out_idx, double alpha, double beta, bool rkc,
                        bool sr, uint32_t *ctr, hipStream_t st);
hipError_t launch_widen_om(const InstDev *insts, int inst, size_t cells, int b, int s, int i,
                           double *dst, hipStream_t st);
hipError_t launch_pack_om(const InstDev *insts, int inst, size_t cells, const double *lo,
                          const double *hi, int b, hipStream_t st);
hipError_t launch_convert_om(const InstDev *insts, int inst, size_t cells, int b, int from, int to,
                             hipStream_t st);
hipError_t launch_init(int prec, const InstDev *insts, int inst, size_t cells,
                       const double *fields, int out_idx, hipStream_t st);
hipError_t launch_moments(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                          double *dst, hipStream_t st);
hipError_t launch_noneq(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int which, double *dst, hipStream_t st);
int totals_blocks();
int energy_rows();
hipError_t launch_energy(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                         int which, double *dst, hipStream_t st);
hipError_t launch_rowsums(const double *src, int nrows, size_t cells, double area, double *part,
                          double *out, hipStream_t st);
hipError_t launch_totals(int prec, const InstDev *insts, int inst, int in_idx, int nq,
                         double area, double *partials, double *out, hipStream_t st);
size_t static_scratch_bytes();
hipError_t static_scratch_init(int *device);
void *static_scratch_get(int dev);
hipError_t launch_totals_static(int prec, const InstDev *insts, int inst, int in_idx, int nq,
                                double area, void *scratch_ptr, double **out, hipStream_t st);
hipError_t launch_widen(int prec, const void *buf, size_t ntot, size_t first, double *dst,
                        size_t n, hipStream_t st);
hipError_t launch_narrow(int prec, const double *src, void *buf, size_t ntot, size_t first,
                         size_t n, hipStream_t st);
hipError_t launch_check(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int *flag, hipStream_t st);
hipError_t launch_dpp_probe(int *out, hipStream_t st);
hipError_t launch_delay(double microseconds, hipStream_t st);
hipError_t launch_copy16(const void *src, void *dst, size_t n16, int grid, int words,
                         hipStream_t st);
}  // namespace dbm

using namespace dbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(DBM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

constexpr int kTilesPerRowStride = 64;  // columns per tile (one per lane)

int tiles_x(int nx) { return (nx + kTilesPerRowStride - 1) / kTilesPerRowStride; }

constexpr int kProbeInts = 640;   // DPP lane-layout probe results

struct Layout {
  size_t sp_off = 0, inst_off = 0, tile_off = 0, part_off = 0, tot_off = 0, flag_off = 0,
         probe_off = 0, ctr_off = 0;
  size_t tile_cap = 0;
  std::vector<size_t> buf_off[3], scratch_off, rref_off, dref_off, orec_off;
  size_t total = 0;
};

int validate(const dbm_config *cfgs, int ninst) {
  if (!cfgs || ninst < 1) return fail(DBM_ERR_ARG, "need at least one configuration");
  for (int k = 0; k < ninst; ++k) {
    const dbm_config &c = cfgs[k];
    const std::string who = "instance " + std::to_string(k) + ": ";
    if (c.nx < 1 || c.ny < 1) return fail(DBM_ERR_ARG, who + "nx, ny must be >= 1");
    if ((double)c.nx * (double)c.ny > (double)(1 << 30))
      return fail(DBM_ERR_ARG, who + "nx*ny above 2^30 cells");
    if (!(c.dx > 0) || !(c.dy > 0) || !(c.dt > 0) || !std::isfinite(c.dx) ||
        !std::isfinite(c.dy) || !std::isfinite(c.dt))
      return fail(DBM_ERR_ARG, who + "dx, dy, dt must be positive and finite");
    if (c.bc_x < 0 || c.bc_x > 2 || c.bc_y < 0 || c.bc_y > 2)
      return fail(DBM_ERR_ARG, who + "unknown boundary condition");
    if (c.nspecies < 1 || c.nspecies > kMaxSpecies || !c.species)
      return fail(DBM_ERR_ARG, who + "nspecies must be 1..16 with a species array");
    if (c.precision < 0 || c.precision > 2 || c.time_scheme < 0 || c.time_scheme > 1 ||
        c.limiter < 0 || c.limiter > 1 || c.force_T_mode < 0 || c.force_T_mode > 1)
      return fail(DBM_ERR_ARG, who + "unknown precision, scheme, limiter or force mode");
    if (!std::isfinite(c.accel[0]) || !std::isfinite(c.accel[1]))
      return fail(DBM_ERR_ARG, who + "non-finite acceleration");
    for (int s = 0; s < c.nspecies; ++s) {
      const dbm_species &sp = c.species[s];
      if (!(sp.m > 0) || !(sp.tau > 0) || !(sp.I >= 0) || !std::isfinite(sp.m) ||
          !std::isfinite(sp.tau) || !std::isfinite(sp.I))
        return fail(DBM_ERR_ARG, who + "species needs m > 0, tau > 0, I >= 0");
    }
    if (c.reaction) {
      const dbm_reaction &r = *c.reaction;
      if (r.fuel < 0 || r.fuel >= c.nspecies || r.oxidiser < 0 || r.oxidiser >= c.nspecies ||
          r.fuel == r.oxidiser)
        return fail(DBM_ERR_ARG, who + "bad fuel/oxidiser indices");
      if (!(r.k_ov >= 0) || !std::isfinite(r.k_ov) || !std::isfinite(r.Ea_over_R) ||
          !std::isfinite(r.Q))
        return fail(DBM_ERR_ARG, who + "bad reaction constants");
      if (r.k_ov > 0)
        for (int s = 1; s < c.nspecies; ++s)
          if (c.species[s].tau != c.species[0].tau)
            return fail(DBM_ERR_UNSUPPORTED,
                        who + "a reaction needs one relaxation time for all species");
    }
    if (c.nchem < 0 || c.nchem > DBM_MAX_REACTION_STEPS || (c.nchem > 0 && !c.chem))
      return fail(DBM_ERR_ARG, who + "nchem must be 0..4 with a step array");
    bool any_rate = c.reaction && c.reaction->k_ov > 0;
    for (int r = 0; r < c.nchem; ++r) {
      const dbm_reaction_step &st = c.chem[r];
      if (st.fuel < 0 || st.fuel >= c.nspecies || st.oxidiser < 0 || st.oxidiser >= c.nspecies)
        return fail(DBM_ERR_ARG, who + "bad reactant indices in a mechanism step");
      if (!(st.k_ov >= 0) || !std::isfinite(st.k_ov) || !std::isfinite(st.Ea_over_R) ||
          !std::isfinite(st.Q))
        return fail(DBM_ERR_ARG, who + "bad constants in a mechanism step");
      for (int s = 0; s < c.nspecies; ++s)
        if (!std::isfinite(st.a[s])) return fail(DBM_ERR_ARG, who + "non-finite stoichiometry");
      any_rate = any_rate || st.k_ov > 0;
    }
    if (c.nchem > 0 && any_rate)
      for (int s = 1; s < c.nspecies; ++s)
        if (c.species[s].tau != c.species[0].tau)
          return fail(DBM_ERR_UNSUPPORTED,
                      who + "a reaction needs one relaxation time for all species");
    if (k > 0) {
      const dbm_config &c0 = cfgs[0];
      if (c.nspecies != c0.nspecies || c.precision != c0.precision ||
          c.time_scheme != c0.time_scheme || c.limiter != c0.limiter)
        return fail(DBM_ERR_UNSUPPORTED,
                    who + "batched instances must share nspecies, precision, scheme, limiter");
    }
  }
  return DBM_OK;
}

// Bytes per stored value (FP32X: 4-byte value + 2-byte residual) and per
// value of the arithmetic type (plain-path scratch).  An FP32-bulk buffer
// also has room for the A-block residuals of OM storage (S x 4 uint16
// planes after the S x 16 FP32 planes).
size_t esize(const dbm_config &c) {
  return c.precision == DBM_FP32_BULK ? 4 : (c.precision == DBM_FP32X ? 6 : 8);
}
size_t csize(const dbm_config &c) { return c.precision == DBM_FP32_BULK ? 4 : 8; }
// plane stride of the f buffers, in elements
size_t pstride(const dbm_config &c) {
  return plane_stride((size_t)c.nx * c.ny, c.precision == DBM_FP64 ? 8 : 4);
}
// bytes of the values of one buffer, and of the A-block residuals (FP32-bulk)
size_t fvalue_bytes(const dbm_config &c) {
  return (size_t)c.nspecies * kNV * pstride(c) * esize(c);
}
size_t fares_bytes(const dbm_config &c) {
  return c.precision == DBM_FP32_BULK ? (size_t)c.nspecies * 4 * pstride(c) * 2 : 0;
}

void compute_layout(const dbm_config *cfgs, int ninst, Layout &L) {
  const int S = cfgs[0].nspecies;
  size_t off = 0;
  L.sp_off = off;
  off = align_up(off + sizeof(SpeciesDev) * (size_t)ninst * S);
  L.inst_off = off;
  off = align_up(off + sizeof(InstDev) * (size_t)ninst);
  L.tile_cap = 0;
  for (int k = 0; k < ninst; ++k) L.tile_cap += (size_t)tiles_x(cfgs[k].nx) * cfgs[k].ny;
  L.tile_off = off;
  off = align_up(off + sizeof(Tile) * L.tile_cap);
  // per-block partials and totals of the mass/momentum/energy sums (S + 3
  // values) and of the energy diagnostics (energy_rows() per species)
  const size_t nq = std::max<size_t>(S + 3, energy_rows());
  L.part_off = off;
  off = align_up(off + sizeof(double) * (size_t)totals_blocks() * nq);
  L.tot_off = off;
  off = align_up(off + sizeof(double) * std::max<size_t>(S + 3, (size_t)energy_rows() * S));
  L.flag_off = off;
  off = align_up(off + sizeof(int));
  L.probe_off = off;
  off = align_up(off + sizeof(int) * kProbeInts);
  // step counters of stochastic rounding: [0..1] the run's, [2..3] timing launches'
  L.ctr_off = off;
  off = align_up(off + sizeof(uint32_t) * 4);
  for (int b = 0; b < 3; ++b) L.buf_off[b].resize(ninst);
  L.scratch_off.resize(ninst);
  L.rref_off.resize(ninst);
  L.dref_off.resize(ninst);
  L.orec_off.resize(ninst);
  for (int k = 0; k < ninst; ++k) {
    // OM storage references per species and grid row (InstDev::rref, dref)
    L.rref_off[k] = off;
    off = align_up(off + sizeof(double) * (size_t)S * cfgs[k].ny * kRowRef);
    L.dref_off[k] = off;
    off = align_up(off + sizeof(float) * (size_t)S * (cfgs[k].ny + 4) * 4);
    L.orec_off[k] = off;
    off = align_up(off + sizeof(uint32_t) * (size_t)S * cfgs[k].ny * kRowRec);
  }
  for (int k = 0; k < ninst; ++k) {
    const size_t cells = (size_t)cfgs[k].nx * cfgs[k].ny;
    const size_t fbytes = fvalue_bytes(cfgs[k]) + fares_bytes(cfgs[k]);
    for (int b = 0; b < 3; ++b) {
      L.buf_off[b][k] = off;
      off = align_up(off + fbytes);
    }
    size_t per_cell = std::max<size_t>((size_t)S * kNV * csize(cfgs[k]), 12 * sizeof(double));
    per_cell = std::max<size_t>(per_cell, (size_t)(S + 3) * sizeof(double));
    L.scratch_off[k] = off;
    off = align_up(off + per_cell * cells);
  }
  L.total = off;
}

struct TuneKey {
  int prec, S, lim, scheme, bucket, ninst, split_opt;
  bool operator<(const TuneKey &o) const {
    return std::tie(prec, S, lim, scheme, bucket, ninst, split_opt) <
           std::tie(o.prec, o.S, o.lim, o.scheme, o.bucket, o.ninst, o.split_opt);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;  // -> (rows, form)
std::mutex g_probe_mu;
int g_probe_state = 0;  // 0 unknown, 1 ok, -1 failed
int g_probe_om = 0;     // broadcasts of the OM halo transform: 1 ok, -1 failed

}  // namespace

struct dbm_s {
  int ninst = 0, S = 0, scheme = 0, lim = 0;
  bool fp32 = false;     // FP32-bulk
  int prec = DBM_FP64;  // DBM_FP64 | DBM_FP32_BULK | DBM_FP32X
  int sr = 0;           // DBM_OPT_ROUNDING: 1 stochastic rounding of FP32 stores
  int om_opt = 0;       // DBM_OPT_STORAGE: 0 OM storage where available, 1 f itself,
                        // 2 OM storage with A-block residuals where available
  int device = 0;       // device current at dbm_create
  bool om = false;      // the buffers (every instance) hold OM storage
  bool ares = false;    // ... with A-block residuals
  std::vector<SpeciesDev> tabs;  // host copy of the species tables
  // OM storage reference per instance and grid row: n_ref^s [s * ny + y] and
  // T_ref [y]; rowref[k]: instance k's references differ between rows (else
  // one reference serves the grid)
  std::vector<std::vector<double>> ref_n, ref_T;
  std::vector<char> rowref;
  // stage-kernel form of the storage: 0 f itself, 1 OM storage with one
  // reference per grid, 2 with references per row (some instance needs them)
  int om_mode() const {
    if (!om) return 0;
    for (char r : rowref)
      if (r) return 2;
    return 1;
  }
  std::vector<dbm_config> cfg;
  std::vector<std::vector<dbm_species>> species;
  std::vector<dbm_reaction> reaction;
  std::vector<std::vector<dbm_reaction_step>> chem;
  hipStream_t stream = nullptr, cap = nullptr;
  char *ws = nullptr;
  Layout L;
  std::vector<InstDev> inst;
  int cur = 0;
  int path = 0, use_graph = 1, tile_rows_opt = 0, check_every = 0, batch_mode = 0,
      graph_chunk = 256;
  bool fused_ok = false;
  int rows = 0;  // rows per tile in use (0 = not tuned yet)
  int split_opt = 0;    // DBM_OPT_SPLIT: 0 tuned, 1 full form, 2 split form
  bool split = false;   // form in use
  bool pipe = false;    // row pipelining in use (FP32 full form)
  int pipe_opt = 0;     // DBM_OPT_PIPELINE: 0 tuned, 1 off, 2 on
  bool cw = false;      // chain wavefront in use (full form, S <= 3)
  bool drain = true;    // OM storage: every other row waits for its refill at once
  int drain_opt = 0;    // DBM_OPT_DRAIN: 0 tuned with the tile rows (on when the
                        // rows are set), 1 off, 2 on
  int cw_opt = 0;       // DBM_OPT_CHAIN_WAVE: 0 tuned, 1 off, 2 on
  std::vector<Tile> tiles;
  std::vector<int> tile_begin;
  // workgroups resident on the device, per form
  int resident = 0, resident_split = 0, resident_cw = 0, resident_om = 0, resident_om_cw = 0,
      resident_ar = 0, resident_ar_cw = 0;
  int grid_cap() const {
    if (om && ares) return cw ? resident_ar_cw : resident_ar;
    if (om) return cw ? resident_om_cw : resident_om;
    return split ? resident_split : (cw ? resident_cw : resident);
  }
  // resident workgroups of the chain-wavefront form of the storage in use
  int cw_resident() const {
    if (om && ares) return resident_ar_cw;
    return om ? resident_om_cw : resident_cw;
  }
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  long long since_check = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  const InstDev *d_inst() const { return (const InstDev *)(ws + L.inst_off); }
  uint32_t *d_ctr(bool timing) const { return (uint32_t *)(ws + L.ctr_off) + (timing ? 2 : 0); }
  const Tile *d_tiles() const { return (const Tile *)(ws + L.tile_off); }
  size_t cells(int k) const { return (size_t)cfg[k].nx * cfg[k].ny; }
  size_t ps(int k) const { return pstride(cfg[k]); }
};

namespace {

void clear_graphs(dbm_handle h) {
  for (auto &kv : h->graphs) hipGraphExecDestroy(kv.second);
  h->graphs.clear();
}

bool use_fused(dbm_handle h) { return h->path == 0 && h->fused_ok; }

void build_tiles(dbm_handle h, int rows) {
  h->tiles.clear();
  h->tile_begin.assign(h->ninst + 1, 0);
  for (int k = 0; k < h->ninst; ++k) {
    h->tile_begin[k] = (int)h->tiles.size();
    const int nx = h->cfg[k].nx, ny = h->cfg[k].ny;
    const int r = std::max(1, std::min(rows, ny));
    for (int y0 = 0; y0 < ny; y0 += r)
      for (int tx = 0; tx < tiles_x(nx); ++tx)
        h->tiles.push_back(Tile{k, tx * kTilesPerRowStride, y0, std::min(r, ny - y0)});
  }
  h->tile_begin[h->ninst] = (int)h->tiles.size();
}

int upload_tiles(dbm_handle h) {
  HIPCHK(hipMemcpyAsync(h->ws + h->L.tile_off, h->tiles.data(), sizeof(Tile) * h->tiles.size(),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

// One stage: out = alpha f^n + beta (f + dt L(f)), on stream st.  Timing
// launches (timing) advance a step counter of their own, so that they leave
// the run's stochastic rounding unchanged.
int enqueue_stage(dbm_handle h, int in_idx, int fn_idx, int out_idx, double alpha, double beta,
                  bool rkc, hipStream_t st, bool timing = false) {
  uint32_t *ctr = h->d_ctr(timing);
  if (use_fused(h)) {
    if (h->batch_mode == 0) {
      const int nt = (int)h->tiles.size();
      const int grid = std::max(1, std::min(nt, h->grid_cap()));
      HIPCHK(launch_fused(h->prec, h->S, h->lim, rkc, h->split, h->pipe, h->sr != 0, h->cw,
                          h->om_mode(), h->om && h->ares, h->om && h->drain, ctr, h->d_inst(),
                          h->d_tiles(), nt, grid, in_idx, fn_idx, out_idx, alpha, beta, st));
    } else {
      for (int k = 0; k < h->ninst; ++k) {
        const int b = h->tile_begin[k], nt = h->tile_begin[k + 1] - b;
        const int grid = std::max(1, std::min(nt, h->grid_cap()));
        HIPCHK(launch_fused(h->prec, h->S, h->lim, rkc, h->split, h->pipe, h->sr != 0, h->cw,
                            h->om_mode(), h->om && h->ares, h->om && h->drain, ctr, h->d_inst(),
                            h->d_tiles() + b, nt, grid, in_idx, fn_idx, out_idx, alpha, beta,
                            st));
      }
    }
  } else {
    for (int k = 0; k < h->ninst; ++k)
      HIPCHK(launch_plain(h->prec, h->d_inst(), k, h->cells(k), h->S, in_idx, fn_idx, out_idx,
                          alpha, beta, rkc, h->sr != 0, ctr, st));
  }
  return DBM_OK;
}

// Enqueue one full time step starting from state buffer `parity`.
int enqueue_step(dbm_handle h, int &parity, hipStream_t st) {
  int rc;
  if (h->scheme == DBM_EULER) {
    rc = enqueue_stage(h, parity, parity, 1 - parity, 0.0, 1.0, false, st);
    if (rc) return rc;
    parity = 1 - parity;
  } else {  // Shu-Osher TVD-RK3; stage 3 overwrites f^n in place (centre reads only)
    if ((rc = enqueue_stage(h, 0, 0, 1, 0.0, 1.0, false, st))) return rc;
    if ((rc = enqueue_stage(h, 1, 0, 2, 0.75, 0.25, true, st))) return rc;
    if ((rc = enqueue_stage(h, 2, 0, 0, 1.0 / 3.0, 2.0 / 3.0, true, st))) return rc;
    parity = 0;
  }
  return DBM_OK;
}

// The stage launch a step is made of (Euler) or that dominates it (RK3,
// stages 2-3), writing only a spare buffer.
int enqueue_timed_stage(dbm_handle h, hipStream_t st) {
  if (h->scheme == DBM_EULER)
    return enqueue_stage(h, h->cur, h->cur, 1 - h->cur, 0.0, 1.0, false, st, true);
  return enqueue_stage(h, 1, 0, 2, 0.75, 0.25, true, st, true);
}

// Mean launch time over reps back-to-back launches; med (optional) gets the
// median, which the autotuner compares (robust to an occasional slow launch).
int time_stage(dbm_handle h, int reps, double *ms, double *med = nullptr) {
  // Fill the queue behind a short delay kernel so that back-to-back launches
  // are timed, not the host's submission rate.
  HIPCHK(launch_delay(50.0 + 25.0 * reps, h->stream));
  // events released on every return path
  struct Events {
    std::vector<hipEvent_t> v;
    ~Events() {
      for (auto e : v)
        if (e) hipEventDestroy(e);
    }
  } evs;
  evs.v.assign(2 * reps, nullptr);
  std::vector<hipEvent_t> &ev = evs.v;
  for (auto &e : ev) HIPCHK(hipEventCreate(&e));
  int rc = DBM_OK;
  for (int r = 0; r < reps && !rc; ++r) {
    HIPCHK(hipEventRecord(ev[2 * r], h->stream));
    rc = enqueue_timed_stage(h, h->stream);
    HIPCHK(hipEventRecord(ev[2 * r + 1], h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  double tot = 0.0;
  std::vector<double> ts;
  for (int r = 0; r < reps && !rc; ++r) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]));
    tot += t;
    ts.push_back(t);
  }
  if (rc) return rc;
  *ms = tot / reps;
  if (med) {
    std::sort(ts.begin(), ts.end());
    *med = ts[ts.size() / 2];
  }
  return DBM_OK;
}

int ensure_tuned(dbm_handle h) {
  if (!use_fused(h)) return DBM_OK;
  int want = h->tile_rows_opt;
  // form: the split form only when asked for (measured slower than the
  // full form on every workload here, so the tuner does not try it)
  int form = h->split_opt == 2 ? 1 : 0;
  const bool tune_form = false;
  int maxny = 1;
  size_t tot = 0;
  for (int k = 0; k < h->ninst; ++k) {
    maxny = std::max(maxny, h->cfg[k].ny);
    tot += h->cells(k);
  }
  const TuneKey key{h->prec, h->S, h->lim, h->scheme,
                    (int)std::lround(std::log2((double)tot + 1.0)), h->ninst,
                    (((((h->split_opt * 3 + h->pipe_opt) * 3 + h->cw_opt) * 2 + h->sr) * 3 +
                      h->om_mode()) * 2 + (h->ares ? 1 : 0)) * 3 + h->drain_opt};
  if (want <= 0) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      want = it->second.first;
      form = it->second.second;
    }
  }
  if (want <= 0) {
    if (h->scheme == DBM_TVD_RK3) {  // give the timed stage realistic inputs
      for (int k = 0; k < h->ninst; ++k)
        HIPCHK(hipMemcpyAsync(h->inst[k].buf[1], h->inst[k].buf[0],
                              fvalue_bytes(h->cfg[k]) + fares_bytes(h->cfg[k]),
                              hipMemcpyDeviceToDevice, h->stream));
    }
    const int cands[] = {1, 2, 4, 8, 16, 32, 64, 128, 256, 512};
    double best = 1e300;
    int best_rows = 1, best_form = form;
    for (int f = 0; f < 2; ++f) {
      if (!tune_form && f != form) continue;
      h->split = f == 1;
      // the row pipeline (pp 1) exists for the FP32 full form, the chain
      // wavefront (pp 2) for the full form with S <= 3
      const bool can_pipe = h->fp32 && f == 0 && !h->om;
      const bool can_cw = f == 0 && h->S <= 3 && h->cw_resident() > 0;
      for (int pp = 0; pp < 3; ++pp) {
        if (pp == 1 && (!can_pipe || h->pipe_opt == 1)) continue;
        if (pp == 2 && (!can_cw || h->cw_opt == 1)) continue;
        if (h->pipe_opt == 2 && can_pipe && pp != 1) continue;
        if (h->cw_opt == 2 && can_cw && pp != 2) continue;
        h->pipe = pp == 1;
        h->cw = pp == 2;
        for (int r : cands) {
          if (r > 2 * maxny && r > 1) break;
          build_tiles(h, r);
          int rc = upload_tiles(h);
          if (rc) return rc;
          // OM storage: the refills kept in flight, or every other row's
          // waited for at once (fewer loads in flight; the faster of the two
          // depends on the workload)
          for (int dr = 1; dr >= (h->om ? 0 : 1); --dr) {
            if (h->om && h->drain_opt == 2 - dr) continue;   // the form not asked for
            h->drain = dr == 1;
            double ms = 0.0;
            if ((rc = time_stage(h, 1, &ms))) return rc;  // warm-up
            if ((rc = time_stage(h, 3, &ms))) return rc;
            // short launches: about 1 ms of launches, compared by the median
            const int reps =
                ms < 0.1 ? std::min(48, std::max(5, (int)(1.0 / std::max(ms, 1e-3)))) : 3;
            if (reps > 3) {
              double mean = 0.0;
              if ((rc = time_stage(h, reps, &mean, &ms))) return rc;
            }
            if (ms < best) {
              best = ms;
              best_rows = r;
              best_form = f | (pp == 1 ? 2 : 0) | (pp == 2 ? 4 : 0) | (dr ? 8 : 0);
            }
          }
        }
      }
    }
    want = best_rows;
    form = best_form;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = std::make_pair(want, form);
  }
  if (h->tile_rows_opt > 0) {  // fixed rows: the form and pipeline the options ask for
    form = h->split_opt == 2 ? 1 : 0;
    if (form == 0 && h->fp32 && h->pipe_opt == 2) form = 2;
    if (form == 0 && h->cw_opt == 2 && h->S <= 3 &&
        h->cw_resident() > 0)
      form = 4;
    if (h->drain_opt != 1) form |= 8;  // OM storage: every other row's refill waited for
  }
  if (want != h->rows || h->tiles.empty() || h->split != ((form & 1) != 0) ||
      h->pipe != ((form & 2) != 0) || h->cw != ((form & 4) != 0) ||
      h->drain != ((form & 8) != 0)) {
    h->split = (form & 1) != 0;
    h->pipe = (form & 2) != 0;
    h->cw = (form & 4) != 0;
    h->drain = (form & 8) != 0;
    build_tiles(h, want);
    int rc = upload_tiles(h);
    if (rc) return rc;
    h->rows = want;
    clear_graphs(h);
  }
  return DBM_OK;
}

int get_graph(dbm_handle h, int parity, int nsteps, hipGraphExec_t *out) {
  auto key = std::make_pair(parity, nsteps);
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) {
    *out = it->second;
    return DBM_OK;
  }
  HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  int p = parity, rc = DBM_OK;
  for (int s = 0; s < nsteps && !rc; ++s) rc = enqueue_step(h, p, h->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(DBM_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess)
    return fail(DBM_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
  h->graphs[key] = ex;
  *out = ex;
  return DBM_OK;
}

int check_state(dbm_handle h) {
  int *flag = (int *)(h->ws + h->L.flag_off);
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), h->stream));
  for (int k = 0; k < h->ninst; ++k)
    HIPCHK(launch_check(h->prec, h->d_inst(), k, h->cells(k), h->cur, flag, h->stream));
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (hflag) return fail(DBM_ERR_NONFINITE, "non-finite value or negative density in f");
  return DBM_OK;
}

int run_probe(dbm_handle h) {
  std::lock_guard<std::mutex> g(g_probe_mu);
  if (g_probe_state != 0) return DBM_OK;
  int *d = (int *)(h->ws + h->L.probe_off);
  int out[kProbeInts];
  HIPCHK(launch_dpp_probe(d, h->stream));
  HIPCHK(hipMemcpyAsync(out, d, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  bool ok = true;
  for (int rep = 0; rep < 2; ++rep)
    for (int l = 0; l < 64; ++l) {
      const int shr = out[128 * rep + l], shl = out[128 * rep + 64 + l];
      ok &= shr == (l == 0 ? -1 : l - 1);
      ok &= shl == (l == 63 ? -1 : l + 1);
      // guard-lane forms of lane value l+1: lane 0 / lane 63 read 0
      const int gr = out[256 + 128 * rep + l], gl = out[320 + 128 * rep + l];
      ok &= gr == (l == 0 ? 0 : l);
      ok &= gl == (l == 63 ? 0 : l + 2);
    }
  g_probe_state = ok ? 1 : -1;
  bool om_ok = true;   // row and quad broadcasts of the OM halo transform
  for (int l = 0; l < 64; ++l) {
    om_ok &= out[512 + l] == 16 * (l / 16) + 4;
    om_ok &= out[576 + l] == 4 * (l / 4) + 2;
  }
  g_probe_om = om_ok ? 1 : -1;
  return DBM_OK;
}

// Whether the options ask for OM storage: FP32-bulk on the one-pass path in
// its full form without the row pipeline, OM storage not switched off, and
// the halo transform's lane broadcasts verified on this device.
bool want_om(dbm_handle h) {
  return h->prec == DBM_FP32_BULK && h->om_opt != 1 && use_fused(h) && h->split_opt != 2 &&
         h->pipe_opt != 2 && g_probe_om > 0 && h->resident_om > 0;
}
// ... and with A-block residuals (storage option 2; round to nearest).
bool want_ares(dbm_handle h) {
  return want_om(h) && h->om_opt == 2 && h->sr == 0 && h->resident_ar > 0;
}
// representation of the buffers: 0 f, 1 OM storage, 2 with A-block residuals
int storage_mode(bool om, bool ares) { return om ? (ares ? 2 : 1) : 0; }

int upload_inst(dbm_handle h) {
  for (auto &d : h->inst) {
    d.om = h->om ? 1 : 0;
    d.ares = h->om && h->ares ? 1 : 0;
  }
  HIPCHK(hipMemcpyAsync(h->ws + h->L.inst_off, h->inst.data(), sizeof(InstDev) * h->ninst,
                        hipMemcpyHostToDevice, h->stream));
  return DBM_OK;
}

int upload_tables(dbm_handle h, int inst) {
  const size_t off = h->L.sp_off + sizeof(SpeciesDev) * (size_t)inst * h->S;
  HIPCHK(hipMemcpyAsync(h->ws + off, h->tabs.data() + (size_t)inst * h->S,
                        sizeof(SpeciesDev) * h->S, hipMemcpyHostToDevice, h->stream));
  return DBM_OK;
}

// Bring every instance's current buffer into the representation the options
// ask for (FP32 f <-> OM storage, in place; FP64 arithmetic per cell).
int sync_storage(dbm_handle h) {
  const bool want = want_om(h), want_ar = want_ares(h);
  const int from = storage_mode(h->om, h->ares), to = storage_mode(want, want_ar);
  if (from == to) return DBM_OK;
  for (int k = 0; k < h->ninst; ++k)
    HIPCHK(launch_convert_om(h->d_inst(), k, h->cells(k), h->cur, from, to, h->stream));
  h->om = want;
  h->ares = want_ar;
  int rc = upload_inst(h);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  h->rows = 0;
  h->tiles.clear();
  clear_graphs(h);
  return DBM_OK;
}

// y-boundary map of the host (the kernels' map_y): the grid row that holds
// row r, and whether it is reflected.
int host_map_y(int r, int ny, int bc, bool &flip) {
  flip = false;
  if (r >= 0 && r < ny) return r;
  if (bc == BC_PERIODIC) return ((r % ny) + ny) % ny;
  if (bc == BC_OUTFLOW) return r < 0 ? 0 : ny - 1;
  // specular wall: reflection about the wall face, repeated if needed
  const int p = 2 * ny;
  int q = ((r % p) + p) % p;
  if (q >= ny) {
    q = p - 1 - q;
    flip = true;
  }
  return q;
}

// OM storage reference of instance inst, per grid row: an equilibrium at
// rest with the row means of each species' density and of the temperature
// of the state being set (n_row [s * ny + y], T_row [y]; non-finite or
// negative entries are taken as 0: no offset).  Builds and uploads the FP64
// references with their A-block moments and the FP32 differences between
// consecutive rows, one per velocity group (an equilibrium at rest has one
// value per group), rows outside the grid as the y boundary maps them, and
// the one-pass kernel's per-row records of both (InstDev::orec).
int set_om_reference(dbm_handle h, int inst, const std::vector<double> &n_row,
                     const std::vector<double> &T_row) {
  const int S = h->S, ny = h->cfg[inst].ny, bcy = h->cfg[inst].bc_y;
  std::vector<double> n(n_row), T(T_row);
  for (auto &v : n)
    if (!std::isfinite(v) || v < 0.0) v = 0.0;
  for (auto &v : T)
    if (!std::isfinite(v) || v < 0.0) v = 0.0;
  // References per row only where the rows differ by more than 1e-3 of the
  // mean (density of a species or temperature); otherwise every row takes
  // the grid's mean, and the stage kernel's form without the per-row terms
  // runs.
  auto spread = [&](const double *v) {
    double m = 0.0, d = 0.0;
    for (int y = 0; y < ny; ++y) m += v[y] / ny;
    for (int y = 0; y < ny; ++y) d = std::fmax(d, std::fabs(v[y] - m));
    return std::make_pair(m, d > 1e-3 * m);
  };
  bool rows = spread(T.data()).second;
  for (int s = 0; s < S; ++s) rows = rows || spread(&n[(size_t)s * ny]).second;
  if (!rows) {
    const double tm = spread(T.data()).first;
    for (int y = 0; y < ny; ++y) T[y] = tm;
    for (int s = 0; s < S; ++s) {
      const double nm = spread(&n[(size_t)s * ny]).first;
      for (int y = 0; y < ny; ++y) n[(size_t)s * ny + y] = nm;
    }
  }
  if ((h->rowref[inst] != 0) != rows) {   // another kernel form: graphs are stale
    h->rowref[inst] = rows ? 1 : 0;
    clear_graphs(h);
  }
  std::vector<double> rr((size_t)S * ny * kRowRef);
  std::vector<float> dr((size_t)S * (ny + 4) * 4);
  std::vector<uint32_t> rec((size_t)S * ny * kRowRec, 0u);
  for (int s = 0; s < S; ++s) {
    const SpeciesDev &sp = h->tabs[(size_t)inst * S + s];
    for (int y = 0; y < ny; ++y)
      om_reference(sp, n[(size_t)s * ny + y], T[y], &rr[((size_t)s * ny + y) * kRowRef]);
    // fref of group g at row r as the boundary map sees it (a reflected row
    // is the mirrored row, whose groups are unchanged by the reflection)
    auto fref = [&](int r, int g) {
      bool flip;
      const int q = host_map_y(r, ny, bcy, flip);
      return rr[((size_t)s * ny + q) * kRowRef + 4 * g];
    };
    for (int r = -2; r <= ny + 1; ++r)
      for (int g = 0; g < 4; ++g)
        dr[((size_t)s * (ny + 4) + r + 2) * 4 + g] = (float)(fref(r + 1, g) - fref(r, g));
    for (int y = 0; y < ny; ++y) {
      uint32_t *w = &rec[((size_t)s * ny + y) * kRowRec];
      std::memcpy(w, &dr[((size_t)s * (ny + 4) + y + 2) * 4], sizeof(float) * 8);
      std::memcpy(w + 8, &rr[((size_t)s * ny + y) * kRowRef + kNV], sizeof(double) * 4);
      if (y + 2 < ny) std::memcpy(w + 16, &rr[((size_t)s * ny + y + 2) * kRowRef + kNV],
                                  sizeof(double) * 2);
    }
  }
  // the single reference's moments also sit in the species tables (the
  // stage kernel's form without per-row references reads them there)
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < 4; ++j)
      h->tabs[(size_t)inst * S + s].sref[j] = rr[((size_t)s * ny) * kRowRef + kNV + j];
  if (int rc = upload_tables(h, inst)) return rc;
  HIPCHK(hipMemcpyAsync(h->ws + h->L.rref_off[inst], rr.data(), sizeof(double) * rr.size(),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->ws + h->L.dref_off[inst], dr.data(), sizeof(float) * dr.size(),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->ws + h->L.orec_off[inst], rec.data(), sizeof(uint32_t) * rec.size(),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->ref_n[inst] = n;
  h->ref_T[inst] = T;
  return DBM_OK;
}

// Checkpoint blob: this header, then the instance's current f buffer as
// stored (S x 16 planes of stride ps in the storage precision, FP32X with its
// residual planes, OM storage with its A-block residuals when in use), so
// that a restart continues bit for bit.
struct StateHeader {
  uint64_t magic;
  int32_t prec, om, S, nx, ny, sr;
  uint64_t buffer_bytes;
  uint32_t ctr[2];
};
// ... followed by the OM references of the rows, (S + 1) x ny FP64 values
// (n_ref^s per row, then T_ref per row), then the buffer.
size_t state_ref_bytes(dbm_handle h, int inst) {
  return sizeof(double) * (size_t)(h->S + 1) * h->cfg[inst].ny;
}
constexpr uint64_t kStateMagic = 0x4554415453424D44ULL;   // "DBMSTATE" in little-endian bytes
size_t buffer_bytes(dbm_handle h, int inst) {
  return fvalue_bytes(h->cfg[inst]) + (h->om && h->ares ? fares_bytes(h->cfg[inst]) : 0);
}

int reset_counters(dbm_handle h) {
  HIPCHK(hipMemsetAsync(h->ws + h->L.ctr_off, 0, sizeof(uint32_t) * 4, h->stream));
  return DBM_OK;
}

int check_inst(dbm_handle h, int inst) {
  if (!h) return fail(DBM_ERR_ARG, "null handle");
  if (inst < 0 || inst >= h->ninst) return fail(DBM_ERR_ARG, "instance index out of range");
  return DBM_OK;
}

}  // namespace

extern "C" {

const char *dbm_last_error(void) { return g_err.c_str(); }

size_t dbm_workspace_bytes(const dbm_config *cfgs, int ninst) {
  if (validate(cfgs, ninst) != DBM_OK) return 0;
  Layout L;
  compute_layout(cfgs, ninst, L);
  return L.total;
}

int dbm_create(const dbm_config *cfgs, int ninst, void *hip_stream, void *dev_workspace,
               size_t ws_bytes, dbm_handle *out) {
  if (!out) return fail(DBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(cfgs, ninst);
  if (rc) return rc;
  Layout L;
  compute_layout(cfgs, ninst, L);
  std::vector<SpeciesDev> tabs((size_t)ninst * cfgs[0].nspecies);
  for (int k = 0; k < ninst; ++k)
    for (int s = 0; s < cfgs[k].nspecies; ++s) {
      std::string err;
      rc = build_species(cfgs[k].species[s], cfgs[k], tabs[(size_t)k * cfgs[0].nspecies + s], err);
      if (rc)
        return fail(rc, "instance " + std::to_string(k) + " species " + std::to_string(s) +
                            ": " + err);
    }
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0)
    return fail(DBM_ERR_WORKSPACE, "workspace is NULL or not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(DBM_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total) +
                                       " bytes");
  dbm_s *h = new dbm_s();
  h->tabs = tabs;
  h->ref_n.resize(ninst);
  h->ref_T.resize(ninst);
  h->rowref.assign(ninst, 0);
  for (int k = 0; k < ninst; ++k) {
    h->ref_n[k].assign((size_t)cfgs[0].nspecies * cfgs[k].ny, 0.0);
    h->ref_T[k].assign((size_t)cfgs[k].ny, 0.0);
  }
  h->ninst = ninst;
  h->S = cfgs[0].nspecies;
  h->fp32 = cfgs[0].precision == DBM_FP32_BULK;
  h->prec = cfgs[0].precision;
  h->scheme = cfgs[0].time_scheme;
  h->lim = cfgs[0].limiter;
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char *)dev_workspace;
  h->L = L;
  h->cfg.assign(cfgs, cfgs + ninst);
  h->species.resize(ninst);
  h->reaction.resize(ninst);
  h->chem.resize(ninst);
  h->fused_ok = h->S <= kMaxFusedSpecies;
  for (int k = 0; k < ninst; ++k) {
    h->species[k].assign(cfgs[k].species, cfgs[k].species + cfgs[k].nspecies);
    h->cfg[k].species = h->species[k].data();
    if (cfgs[k].reaction) {
      h->reaction[k] = *cfgs[k].reaction;
      h->cfg[k].reaction = &h->reaction[k];
    } else {
      h->cfg[k].reaction = nullptr;
    }
    h->chem[k].assign(cfgs[k].chem, cfgs[k].chem + cfgs[k].nchem);
    h->cfg[k].chem = h->chem[k].empty() ? nullptr : h->chem[k].data();
    if (cfgs[k].bc_x == DBM_BC_WALL) h->fused_ok = false;
    // the one-pass kernel addresses one species' 16 planes with 32-bit offsets
    if ((double)kNV * (double)pstride(cfgs[k]) * (h->prec == DBM_FP64 ? 8.0 : 4.0) >=
        4294967296.0)
      h->fused_ok = false;
    InstDev d;
    std::memset(&d, 0, sizeof(d));
    for (int b = 0; b < 3; ++b) d.buf[b] = h->ws + L.buf_off[b][k];
    d.ps = pstride(cfgs[k]);
    d.scratch = h->ws + L.scratch_off[k];
    d.sp = (const SpeciesDev *)(h->ws + L.sp_off) + (size_t)k * h->S;
    d.rref = (const double *)(h->ws + L.rref_off[k]);
    d.dref = (const float *)(h->ws + L.dref_off[k]);
    d.orec = (const uint32_t *)(h->ws + L.orec_off[k]);
    d.nx = cfgs[k].nx;
    d.ny = cfgs[k].ny;
    d.bcx = cfgs[k].bc_x;
    d.bcy = cfgs[k].bc_y;
    d.S = h->S;
    // chemistry: the mechanism's steps, or the one-step reaction as step 0
    auto add_step = [&](int fuel, int oxid, double kr, double ea, double q, const double *a) {
      const int r = d.nreact++;
      d.rfuel[r] = fuel;
      d.roxid[r] = oxid;
      d.rk[r] = kr;
      d.rEa[r] = ea;
      d.rQ2[r] = 2.0 * q;
      d.rdK[r] = 0.0;
      for (int s = 0; s < h->S; ++s) {
        d.ra[r][s] = a[s];
        d.rneg[r][s] = a[s] < 0.0 ? -a[s] : 0.0;
        d.rdK[r] += (2.0 + cfgs[k].species[s].I) * a[s];
      }
    };
    if (cfgs[k].nchem > 0) {
      for (int r = 0; r < cfgs[k].nchem; ++r) {
        const dbm_reaction_step &st = cfgs[k].chem[r];
        if (st.k_ov > 0) add_step(st.fuel, st.oxidiser, st.k_ov, st.Ea_over_R, st.Q, st.a);
      }
    } else if (cfgs[k].reaction && cfgs[k].reaction->k_ov > 0) {
      const dbm_reaction *r = cfgs[k].reaction;
      double a[kMaxSpecies] = {0};
      for (int s = 0; s < h->S; ++s) a[s] = cfgs[k].species[s].a_stoich;
      add_step(r->fuel, r->oxidiser, r->k_ov, r->Ea_over_R, r->Q, a);
    }
    d.force = (cfgs[k].accel[0] != 0.0 || cfgs[k].accel[1] != 0.0) ? 1 : 0;
    d.fmode = cfgs[k].force_T_mode;
    d.ax = cfgs[k].accel[0];
    d.ay = cfgs[k].accel[1];
    d.dt = cfgs[k].dt;
    d.dx = cfgs[k].dx;
    d.dy = cfgs[k].dy;
    d.lim = cfgs[k].limiter;
    h->inst.push_back(d);
  }
  auto bail = [&](int code) {
    if (h->cap) hipStreamDestroy(h->cap);
    if (h->ev0) hipEventDestroy(h->ev0);
    if (h->ev1) hipEventDestroy(h->ev1);
    delete h;
    return code;
  };
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreate(&h->ev0)) != hipSuccess || (e = hipEventCreate(&h->ev1)) != hipSuccess)
    return bail(fail(DBM_ERR_HIP, std::string("stream/event creation: ") + hipGetErrorString(e)));
  if ((e = hipMemcpyAsync(h->ws + L.sp_off, tabs.data(), sizeof(SpeciesDev) * tabs.size(),
                          hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(h->ws + L.inst_off, h->inst.data(), sizeof(InstDev) * ninst,
                          hipMemcpyHostToDevice, h->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(h->stream)) != hipSuccess)
    return bail(fail(DBM_ERR_HIP, std::string("table upload: ") + hipGetErrorString(e)));
  // OM storage references: none (zero) until the fields are set
  if (h->prec == DBM_FP32_BULK)
    for (int k = 0; k < ninst; ++k)
      if ((rc = set_om_reference(h, k, h->ref_n[k], h->ref_T[k]))) return bail(rc);
  if ((rc = run_probe(h))) return bail(rc);
  // the fixed scratch of dbm_noneq_totals_noalloc on this device, located now
  if ((e = static_scratch_init(&h->device)) != hipSuccess)
    return bail(fail(DBM_ERR_HIP, std::string("scratch symbol: ") + hipGetErrorString(e)));
  if (g_probe_state < 0) h->fused_ok = false;
  if (h->fused_ok) {
    int per_cu = 0, per_cu_split = 0, per_cu_cw = 0, per_cu_om = 0, per_cu_om_cw = 0,
        per_cu_ar = 0, per_cu_ar_cw = 0, dev = 0;
    hipDeviceProp_t prop;
    const bool rk3 = h->scheme == DBM_TVD_RK3;
    auto occ = [&](bool split, bool cw, bool om, bool ar, int *out) {
      return fused_occupancy(h->prec, h->S, h->lim, rk3, split, cw, om, ar, out);
    };
    if ((e = occ(false, false, false, false, &per_cu)) != hipSuccess ||
        (e = occ(true, false, false, false, &per_cu_split)) != hipSuccess ||
        (e = occ(false, true, false, false, &per_cu_cw)) != hipSuccess ||
        (e = occ(false, false, true, false, &per_cu_om)) != hipSuccess ||
        (e = occ(false, true, true, false, &per_cu_om_cw)) != hipSuccess ||
        (e = occ(false, false, true, true, &per_cu_ar)) != hipSuccess ||
        (e = occ(false, true, true, true, &per_cu_ar_cw)) != hipSuccess ||
        (e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
      return bail(fail(DBM_ERR_HIP, std::string("occupancy query: ") + hipGetErrorString(e)));
    auto round_xcd = [](int r) { return std::max(kNumXcd, (r / kNumXcd) * kNumXcd); };
    h->resident = round_xcd(per_cu * prop.multiProcessorCount);
    h->resident_split = round_xcd(per_cu_split * prop.multiProcessorCount);
    h->resident_cw = per_cu_cw > 0 ? round_xcd(per_cu_cw * prop.multiProcessorCount) : 0;
    h->resident_om = per_cu_om > 0 ? round_xcd(per_cu_om * prop.multiProcessorCount) : 0;
    h->resident_om_cw =
        per_cu_om_cw > 0 ? round_xcd(per_cu_om_cw * prop.multiProcessorCount) : 0;
    h->resident_ar = per_cu_ar > 0 ? round_xcd(per_cu_ar * prop.multiProcessorCount) : 0;
    h->resident_ar_cw =
        per_cu_ar_cw > 0 ? round_xcd(per_cu_ar_cw * prop.multiProcessorCount) : 0;
  }
  h->om = want_om(h);
  h->ares = want_ares(h);
  if ((rc = upload_inst(h)) || (rc = reset_counters(h))) return bail(rc);
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess)
    return bail(fail(DBM_ERR_HIP, std::string("set-up: ") + hipGetErrorString(e)));
  *out = h;
  return DBM_OK;
}

int dbm_destroy(dbm_handle h) {
  if (!h) return fail(DBM_ERR_ARG, "null handle");
  hipStreamSynchronize(h->stream);
  clear_graphs(h);
  if (h->cap) hipStreamDestroy(h->cap);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  delete h;
  return DBM_OK;
}

int dbm_set_fields(dbm_handle h, int inst, const double *n_sp, const double *ux,
                   const double *uy, const double *T) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!n_sp || !ux || !uy || !T) return fail(DBM_ERR_ARG, "NULL field array");
  const size_t cells = h->cells(inst), S = h->S;
  if (h->prec == DBM_FP32_BULK) {   // OM storage reference: row means of n^s and T, at rest
    const size_t nx = h->cfg[inst].nx, ny = h->cfg[inst].ny;
    std::vector<double> nr(S * ny, 0.0), tr(ny, 0.0);
    for (size_t y = 0; y < ny; ++y) {
      for (size_t s = 0; s < S; ++s) {
        double a = 0.0;
        for (size_t x = 0; x < nx; ++x) a += n_sp[s * cells + y * nx + x];
        nr[s * ny + y] = a / (double)nx;
      }
      double a = 0.0;
      for (size_t x = 0; x < nx; ++x) a += T[y * nx + x];
      tr[y] = a / (double)nx;
    }
    if ((rc = set_om_reference(h, inst, nr, tr))) return rc;
  }
  if ((rc = reset_counters(h))) return rc;
  double *stage = (double *)h->inst[inst].scratch;
  HIPCHK(hipMemcpyAsync(stage, n_sp, sizeof(double) * S * cells, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(stage + S * cells, ux, sizeof(double) * cells, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(stage + (S + 1) * cells, uy, sizeof(double) * cells, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(stage + (S + 2) * cells, T, sizeof(double) * cells, hipMemcpyHostToDevice, h->stream));
  HIPCHK(launch_init(h->prec, h->d_inst(), inst, cells, stage, h->cur, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_set_f(dbm_handle h, int inst, const double *f) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!f) return fail(DBM_ERR_ARG, "NULL f");
  const size_t cells = h->cells(inst), nplanes = (size_t)h->S * kNV, ps = h->ps(inst);
  void *dst = h->inst[inst].buf[h->cur];
  if (h->prec == DBM_FP32_BULK) {
    // OM storage reference from f: row means of each species' density and of
    // the mixture temperature (moments n, j, E of every cell, FP64).
    const int S = h->S;
    const size_t nx = h->cfg[inst].nx, ny = h->cfg[inst].ny;
    std::vector<double> nr((size_t)S * ny, 0.0), tr(ny, 0.0);
    for (size_t c = 0; c < cells; ++c) {
      const size_t y = c / nx;
      double rho = 0, px = 0, py = 0, e = 0, kn = 0;
      for (int s = 0; s < S; ++s) {
        const SpeciesDev &sp = h->tabs[(size_t)inst * S + s];
        double n = 0, jx = 0, jy = 0, E = 0;
        for (int i = 0; i < kNV; ++i) {
          const double v = f[((size_t)s * kNV + i) * cells + c];
          n += v;
          jx += v * sp.M[1 * kNV + i];
          jy += v * sp.M[2 * kNV + i];
          E += v * sp.M[3 * kNV + i];
        }
        nr[(size_t)s * ny + y] += n / (double)nx;
        rho += sp.m * n;
        px += sp.m * jx;
        py += sp.m * jy;
        e += sp.m * E;
        kn += sp.K * n;
      }
      if (rho != 0.0 && kn != 0.0) tr[y] += (e - (px * px + py * py) / rho) / kn / (double)nx;
    }
    if ((rc = set_om_reference(h, inst, nr, tr))) return rc;
  }
  if ((rc = reset_counters(h))) return rc;
  if (h->prec == DBM_FP64) {
    HIPCHK(hipMemcpy2DAsync(dst, sizeof(double) * ps, f, sizeof(double) * cells,
                            sizeof(double) * cells, nplanes, hipMemcpyHostToDevice, h->stream));
  } else if (h->om) {
    // FP64 planes staged in the two spare buffers (each holds S*8 FP64
    // planes of stride ps), then packed into OM storage.
    double *lo = (double *)h->inst[inst].buf[(h->cur + 1) % 3];
    double *hi = (double *)h->inst[inst].buf[(h->cur + 2) % 3];
    const size_t half = nplanes / 2;
    HIPCHK(hipMemcpy2DAsync(lo, sizeof(double) * ps, f, sizeof(double) * cells,
                            sizeof(double) * cells, half, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpy2DAsync(hi, sizeof(double) * ps, f + half * cells, sizeof(double) * cells,
                            sizeof(double) * cells, nplanes - half, hipMemcpyHostToDevice,
                            h->stream));
    HIPCHK(launch_pack_om(h->d_inst(), inst, cells, lo, hi, h->cur, h->stream));
  } else {
    double *stage = (double *)h->inst[inst].scratch;
    for (size_t p = 0; p < nplanes; ++p) {
      HIPCHK(hipMemcpyAsync(stage, f + p * cells, sizeof(double) * cells, hipMemcpyHostToDevice, h->stream));
      HIPCHK(launch_narrow(h->prec, stage, dst, nplanes * ps, p * ps, cells, h->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_get_f(dbm_handle h, int inst, double *f) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!f) return fail(DBM_ERR_ARG, "NULL f");
  const size_t cells = h->cells(inst), nplanes = (size_t)h->S * kNV, ps = h->ps(inst);
  const void *src = h->inst[inst].buf[h->cur];
  if (h->prec == DBM_FP64) {
    HIPCHK(hipMemcpy2DAsync(f, sizeof(double) * cells, src, sizeof(double) * ps,
                            sizeof(double) * cells, nplanes, hipMemcpyDeviceToHost, h->stream));
  } else if (h->om) {
    double *stage = (double *)h->inst[inst].scratch;
    for (size_t p = 0; p < nplanes; ++p) {
      HIPCHK(launch_widen_om(h->d_inst(), inst, cells, h->cur, (int)(p / kNV), (int)(p % kNV),
                             stage, h->stream));
      HIPCHK(hipMemcpyAsync(f + p * cells, stage, sizeof(double) * cells, hipMemcpyDeviceToHost,
                            h->stream));
    }
  } else {
    double *stage = (double *)h->inst[inst].scratch;
    for (size_t p = 0; p < nplanes; ++p) {
      HIPCHK(launch_widen(h->prec, src, nplanes * ps, p * ps, stage, cells, h->stream));
      HIPCHK(hipMemcpyAsync(f + p * cells, stage, sizeof(double) * cells, hipMemcpyDeviceToHost, h->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_step(dbm_handle h, int nsteps) {
  if (!h) return fail(DBM_ERR_ARG, "null handle");
  if (nsteps < 0) return fail(DBM_ERR_ARG, "nsteps < 0");
  int rc = ensure_tuned(h);
  if (rc) return rc;
  while (nsteps > 0) {
    int n = nsteps;
    if (h->check_every > 0) n = (int)std::min<long long>(n, h->check_every - h->since_check);
    if (h->use_graph) {
      int left = n;
      while (left > 0) {
        const int chunk = std::min(left, std::max(1, h->graph_chunk));
        hipGraphExec_t ex;
        if ((rc = get_graph(h, h->cur, chunk, &ex))) return rc;
        HIPCHK(hipGraphLaunch(ex, h->stream));
        if (h->scheme == DBM_EULER && (chunk & 1)) h->cur = 1 - h->cur;
        left -= chunk;
      }
    } else {
      for (int s = 0; s < n; ++s)
        if ((rc = enqueue_step(h, h->cur, h->stream))) return rc;
    }
    nsteps -= n;
    if (h->check_every > 0) {
      h->since_check += n;
      if (h->since_check >= h->check_every) {
        h->since_check = 0;
        if ((rc = check_state(h))) return rc;
      }
    }
  }
  return DBM_OK;
}

int dbm_moments(dbm_handle h, int inst, double *rho_sp, double *ux, double *uy, double *T) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  const size_t cells = h->cells(inst), S = h->S;
  double *stage = (double *)h->inst[inst].scratch;
  HIPCHK(launch_moments(h->prec, h->d_inst(), inst, cells, h->cur, stage, h->stream));
  if (rho_sp) HIPCHK(hipMemcpyAsync(rho_sp, stage, sizeof(double) * S * cells, hipMemcpyDeviceToHost, h->stream));
  if (ux) HIPCHK(hipMemcpyAsync(ux, stage + S * cells, sizeof(double) * cells, hipMemcpyDeviceToHost, h->stream));
  if (uy) HIPCHK(hipMemcpyAsync(uy, stage + (S + 1) * cells, sizeof(double) * cells, hipMemcpyDeviceToHost, h->stream));
  if (T) HIPCHK(hipMemcpyAsync(T, stage + (S + 2) * cells, sizeof(double) * cells, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_noneq_moments(dbm_handle h, int inst, double *delta, double *totals) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  const size_t cells = h->cells(inst);
  double *stage = (double *)h->inst[inst].scratch;
  if (delta) {
    for (int s = 0; s < h->S; ++s) {
      HIPCHK(launch_noneq(h->prec, h->d_inst(), inst, cells, h->cur, s, stage, h->stream));
      HIPCHK(hipMemcpyAsync(delta + (size_t)s * 12 * cells, stage, sizeof(double) * 12 * cells,
                            hipMemcpyDeviceToHost, h->stream));
    }
  }
  if (totals) {
    const int nq = h->S + 3;
    double *part = (double *)(h->ws + h->L.part_off), *tot = (double *)(h->ws + h->L.tot_off);
    HIPCHK(launch_totals(h->prec, h->d_inst(), inst, h->cur, nq,
                         h->cfg[inst].dx * h->cfg[inst].dy, part, tot, h->stream));
    HIPCHK(hipMemcpyAsync(totals, tot, sizeof(double) * nq, hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_noneq_totals_noalloc(dbm_handle h, int inst, double *totals) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!totals) return fail(DBM_ERR_ARG, "NULL totals");
  const int nq = h->S + 3;
  const size_t need = sizeof(double) * ((size_t)totals_blocks() * nq + nq);
  if (need > static_scratch_bytes())
    return fail(DBM_ERR_ARG, "totals need " + std::to_string(need) + " bytes of scratch, more than "
                                 "the fixed " + std::to_string(static_scratch_bytes()));
  void *scr = static_scratch_get(h->device);
  if (!scr) return fail(DBM_ERR_HIP, "fixed scratch not located on the handle's device");
  double *dev_tot = nullptr;
  HIPCHK(launch_totals_static(h->prec, h->d_inst(), inst, h->cur, nq,
                              h->cfg[inst].dx * h->cfg[inst].dy, scr, &dev_tot, h->stream));
  HIPCHK(hipMemcpyAsync(totals, dev_tot, sizeof(double) * nq, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_energy_moments(dbm_handle h, int inst, double *fields, double *totals) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  const size_t cells = h->cells(inst);
  const int nr = energy_rows();
  double *stage = (double *)h->inst[inst].scratch;
  double *part = (double *)(h->ws + h->L.part_off), *tot = (double *)(h->ws + h->L.tot_off);
  const double area = h->cfg[inst].dx * h->cfg[inst].dy;
  for (int s = 0; s < h->S; ++s) {
    HIPCHK(launch_energy(h->prec, h->d_inst(), inst, cells, h->cur, s, stage, h->stream));
    if (fields)
      HIPCHK(hipMemcpyAsync(fields + (size_t)s * nr * cells, stage, sizeof(double) * nr * cells,
                            hipMemcpyDeviceToHost, h->stream));
    if (totals) HIPCHK(launch_rowsums(stage, nr, cells, area, part, tot + (size_t)s * nr, h->stream));
  }
  if (totals)
    HIPCHK(hipMemcpyAsync(totals, tot, sizeof(double) * nr * h->S, hipMemcpyDeviceToHost,
                          h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_set_option(dbm_handle h, int option, int value) {
  if (!h) return fail(DBM_ERR_ARG, "null handle");
  switch (option) {
    case DBM_OPT_PATH:
      if (value < 0 || value > 1) return fail(DBM_ERR_ARG, "path must be 0 or 1");
      if (value == 0 && !h->fused_ok)
        return fail(DBM_ERR_UNSUPPORTED, "fused path needs S <= 4, no x walls, DPP check ok");
      h->path = value;
      break;
    case DBM_OPT_GRAPH: h->use_graph = value ? 1 : 0; break;
    case DBM_OPT_TILE_ROWS:
      if (value < 0 || value > 4096) return fail(DBM_ERR_ARG, "tile rows out of range");
      h->tile_rows_opt = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_CHECK_EVERY:
      if (value < 0) return fail(DBM_ERR_ARG, "check interval < 0");
      h->check_every = value;
      h->since_check = 0;
      break;
    case DBM_OPT_BATCH_MODE:
      if (value < 0 || value > 1) return fail(DBM_ERR_ARG, "batch mode must be 0 or 1");
      h->batch_mode = value;
      break;
    case DBM_OPT_GRAPH_CHUNK:
      if (value < 1 || value > 4096) return fail(DBM_ERR_ARG, "graph chunk out of range");
      h->graph_chunk = value;
      break;
    case DBM_OPT_SPLIT:
      if (value < 0 || value > 2) return fail(DBM_ERR_ARG, "split must be 0, 1 or 2");
      if (value == 2 && h->prec == DBM_FP32X)
        return fail(DBM_ERR_UNSUPPORTED, "the split form has no FP32X storage variant");
      if (value == 2 && h->sr)
        return fail(DBM_ERR_UNSUPPORTED, "the split form has no stochastic rounding");
      if (value == 2 && h->cw_opt == 2)
        return fail(DBM_ERR_UNSUPPORTED, "the chain wavefront excludes the split form");
      h->split_opt = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_PIPELINE:
      if (value < 0 || value > 2) return fail(DBM_ERR_ARG, "pipeline must be 0, 1 or 2");
      if (value == 2 && h->cw_opt == 2)
        return fail(DBM_ERR_UNSUPPORTED, "the chain wavefront replaces the row pipeline");
      h->pipe_opt = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_CHAIN_WAVE:
      if (value < 0 || value > 2) return fail(DBM_ERR_ARG, "chain wave must be 0, 1 or 2");
      if (value == 2 && (h->S > 3 || h->resident_cw == 0 || !h->fused_ok))
        return fail(DBM_ERR_UNSUPPORTED, "the chain wavefront needs the one-pass path and S <= 3");
      if (value == 2 && (h->split_opt == 2 || h->pipe_opt == 2))
        return fail(DBM_ERR_UNSUPPORTED,
                    "the chain wavefront excludes the split form and the row pipeline");
      h->cw_opt = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_DRAIN:
      if (value < 0 || value > 2) return fail(DBM_ERR_ARG, "drain must be 0, 1 or 2");
      h->drain_opt = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_ROUNDING:
      if (value < 0 || value > 1) return fail(DBM_ERR_ARG, "rounding must be 0 or 1");
      if (value == 1 && h->om_opt == 2)
        return fail(DBM_ERR_UNSUPPORTED, "A-block residuals are summed with round to nearest");
      if (value == 1 && h->prec != DBM_FP32_BULK)
        return fail(DBM_ERR_UNSUPPORTED, "stochastic rounding applies to FP32-bulk storage");
      if (value == 1 && h->split_opt == 2)
        return fail(DBM_ERR_UNSUPPORTED, "the split form has no stochastic rounding");
      h->sr = value;
      h->rows = 0;
      h->tiles.clear();
      break;
    case DBM_OPT_STORAGE:
      if (value < 0 || value > 2) return fail(DBM_ERR_ARG, "storage must be 0, 1 or 2");
      if (value == 2 && h->sr)
        return fail(DBM_ERR_UNSUPPORTED, "A-block residuals are summed with round to nearest");
      h->om_opt = value;
      break;
    default: return fail(DBM_ERR_ARG, "unknown or read-only option");
  }
  clear_graphs(h);
  return sync_storage(h);
}

int dbm_get_option(dbm_handle h, int option, int *value) {
  if (!h || !value) return fail(DBM_ERR_ARG, "null handle or value");
  switch (option) {
    case DBM_OPT_PATH: *value = use_fused(h) ? 0 : 1; break;
    case DBM_OPT_GRAPH: *value = h->use_graph; break;
    case DBM_OPT_TILE_ROWS: *value = h->rows; break;
    case DBM_OPT_CHECK_EVERY: *value = h->check_every; break;
    case DBM_OPT_BATCH_MODE: *value = h->batch_mode; break;
    case DBM_OPT_GRAPH_CHUNK: *value = h->graph_chunk; break;
    case DBM_OPT_PERSISTENT: *value = h->grid_cap(); break;
    case DBM_OPT_SPLIT: *value = h->split ? 2 : 1; break;
    case DBM_OPT_PIPELINE: *value = h->pipe ? 2 : 1; break;
    case DBM_OPT_ROUNDING: *value = h->sr; break;
    case DBM_OPT_STORAGE: *value = h->om ? (h->ares ? 2 : 0) : 1; break;
    case DBM_OPT_CHAIN_WAVE: *value = h->cw ? 2 : 1; break;
    case DBM_OPT_DRAIN: *value = h->drain ? 2 : 1; break;
    default: return fail(DBM_ERR_ARG, "unknown option");
  }
  return DBM_OK;
}

int dbm_copy_rate(const void *src, void *dst, size_t bytes, int grid, int words, int reps,
                  void *hip_stream, double *ms_per_copy) {
  if (!src || !dst || !ms_per_copy || reps < 1 || grid < 1 || bytes < 16 || bytes % 16 ||
      ((uintptr_t)src | (uintptr_t)dst) % 16 ||
      !(words == 1 || words == 2 || words == 4 || words == 8))
    return fail(DBM_ERR_ARG, "dbm_copy_rate: bad arguments");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(DBM_ERR_ARG, "dbm_copy_rate: buffers overlap");
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_copy16(src, dst, bytes / 16, grid, words, st);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    e = launch_copy16(src, dst, bytes / 16, grid, words, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (e != hipSuccess) return fail(DBM_ERR_HIP, std::string("dbm_copy_rate: ") + hipGetErrorString(e));
  *ms_per_copy = ms / reps;
  return DBM_OK;
}

size_t dbm_state_bytes(dbm_handle h, int inst) {
  if (check_inst(h, inst)) return 0;
  return sizeof(StateHeader) + state_ref_bytes(h, inst) + buffer_bytes(h, inst);
}

int dbm_save_state(dbm_handle h, int inst, void *dst, size_t bytes) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!dst || bytes < dbm_state_bytes(h, inst)) return fail(DBM_ERR_ARG, "state buffer too small");
  StateHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  hd.magic = kStateMagic;
  hd.prec = h->prec;
  hd.om = storage_mode(h->om, h->ares);
  hd.S = h->S;
  hd.nx = h->cfg[inst].nx;
  hd.ny = h->cfg[inst].ny;
  hd.sr = h->sr;
  hd.buffer_bytes = buffer_bytes(h, inst);
  const size_t rb = state_ref_bytes(h, inst);
  HIPCHK(hipMemcpyAsync(hd.ctr, h->d_ctr(false), sizeof(hd.ctr), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync((char *)dst + sizeof(StateHeader) + rb, h->inst[inst].buf[h->cur],
                        hd.buffer_bytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  std::memcpy(dst, &hd, sizeof(hd));
  const size_t nn = sizeof(double) * h->ref_n[inst].size();
  std::memcpy((char *)dst + sizeof(StateHeader), h->ref_n[inst].data(), nn);
  std::memcpy((char *)dst + sizeof(StateHeader) + nn, h->ref_T[inst].data(), rb - nn);
  return DBM_OK;
}

int dbm_load_state(dbm_handle h, int inst, const void *src, size_t bytes) {
  int rc = check_inst(h, inst);
  if (rc) return rc;
  if (!src || bytes < sizeof(StateHeader)) return fail(DBM_ERR_ARG, "state buffer too small");
  StateHeader hd;
  std::memcpy(&hd, src, sizeof(hd));
  if (hd.magic != kStateMagic || hd.prec != h->prec || hd.om != storage_mode(h->om, h->ares) ||
      hd.S != h->S || hd.nx != h->cfg[inst].nx || hd.ny != h->cfg[inst].ny ||
      hd.buffer_bytes != buffer_bytes(h, inst) || bytes < dbm_state_bytes(h, inst))
    return fail(DBM_ERR_ARG, "state blob does not match this handle's configuration");
  const size_t ny = h->cfg[inst].ny, rb = state_ref_bytes(h, inst);
  std::vector<double> nr((size_t)h->S * ny), tr(ny);
  std::memcpy(nr.data(), (const char *)src + sizeof(StateHeader), sizeof(double) * nr.size());
  std::memcpy(tr.data(), (const char *)src + sizeof(StateHeader) + sizeof(double) * nr.size(),
              sizeof(double) * ny);
  if ((rc = set_om_reference(h, inst, nr, tr))) return rc;
  HIPCHK(hipMemcpyAsync(h->inst[inst].buf[h->cur], (const char *)src + sizeof(StateHeader) + rb,
                        hd.buffer_bytes, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->d_ctr(false), hd.ctr, sizeof(hd.ctr), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return DBM_OK;
}

int dbm_time_stage_kernel(dbm_handle h, int reps, double *ms_per_launch) {
  if (!h || !ms_per_launch || reps < 1) return fail(DBM_ERR_ARG, "bad arguments");
  int rc = ensure_tuned(h);
  if (rc) return rc;
  return time_stage(h, reps, ms_per_launch);
}

}  // extern "C"
