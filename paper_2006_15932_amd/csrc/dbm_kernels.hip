// dbm_kernels.hip -- gfx950 kernels of libdbm.
//
// Data layout in HBM (per instance): three distribution buffers, each
// [S][16][ny][nx] in the storage precision (float for FP32-bulk, double for
// FP64; FP32X: all FP32 parts, then all bf16 parts), x fastest, so every
// velocity plane is a dense 2-D array and a wavefront's 64 lanes read 64
// consecutive cells of one plane per load.  Consecutive planes are InstDev.ps
// elements apart: nx*ny plus a pad of 17 x 256 bytes (plane_stride).
//
// The one-pass stage kernel (k_fused_stage) gives each workgroup a tile of 64
// columns (one per lane, 128-byte aligned) by `rows` rows, one wavefront per
// species, and marches it in +y:
//   * x-neighbours of the NND stencil come from adjacent lanes through DPP
//     whole-wavefront shifts (no LDS, no barriers); the three values beyond
//     the tile's edges that each x-moving plane needs arrive in one compact
//     load per row (36 lanes) and enter the shifts at the edge lanes;
//   * y-neighbours are carried in registers from row to row (three values per
//     plane with a nonzero v_y, one prefetched value for the others), so each
//     value of f is loaded once per tile plus a four-row halo;
//   * per cell, the moments feeding T are summed in FP64, the mixture u, T,
//     reaction and force terms are evaluated in FP64, and f^eq = M^{-1} fhat
//     is formed through the symmetry blocks of M (56 multiply-adds instead of
//     256) before the BGK + source + Runge-Kutta combine and a single store.
// Tiles are taken from a table in an order that keeps x-neighbouring tiles on
// the same XCD (one L2 per XCD) so that the halo columns hit in L2.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <cstdlib>
#include <mutex>

#include "../../include/dbm.h"
#include "dbm_internal.hpp"

// Streaming (non-temporal) stores of the new distribution.
#ifndef DBM_NT_STORE
#define DBM_NT_STORE 1
#endif

namespace dbm {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
// Pointers into HBM read from the instance table are generic; casting them
// to the global address space lets the compiler emit global (not flat)
// memory instructions.
template <typename T> using gptr = const T __attribute__((address_space(1))) *;
template <typename T> using gptr_mut = T __attribute__((address_space(1))) *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(const void *p) {
  return (gptr<T>)(p);
}
template <typename T> __device__ __forceinline__ gptr_mut<T> as_global_mut(void *p) {
  return (gptr_mut<T>)(p);
}

// Species tables are read through the constant address space: wave-uniform,
// read-only, so every access is a scalar load.
#define DBM_CONST __attribute__((address_space(4)))
using SpC = const SpeciesDev DBM_CONST;
__device__ __forceinline__ SpC *as_const(const SpeciesDev *p) { return (SpC *)(p); }

template <typename T> struct Tab;
template <> struct Tab<float> {
  static __device__ __forceinline__ const float DBM_CONST *KA(SpC &s) { return s.KA_f; }
  static __device__ __forceinline__ const float DBM_CONST *KB1(SpC &s) { return s.KB1_f; }
  static __device__ __forceinline__ const float DBM_CONST *KB2(SpC &s) { return s.KB2_f; }
  static __device__ __forceinline__ const float DBM_CONST *KE(SpC &s) { return s.KE_f; }
  static __device__ __forceinline__ const float DBM_CONST *MA(SpC &s) { return s.MA_f; }
  static __device__ __forceinline__ const float DBM_CONST *MB1(SpC &s) { return s.MB1_f; }
  static __device__ __forceinline__ const float DBM_CONST *MB2(SpC &s) { return s.MB2_f; }
  static __device__ __forceinline__ const float DBM_CONST *ME(SpC &s) { return s.ME_f; }
  static __device__ __forceinline__ float cgx(SpC &s, int g) { return s.cgx_f[g]; }
  static __device__ __forceinline__ float cgy(SpC &s, int g) { return s.cgy_f[g]; }
  static __device__ __forceinline__ float omega(SpC &s) { return s.omega_f; }
};
template <> struct Tab<double> {
  static __device__ __forceinline__ const double DBM_CONST *KA(SpC &s) { return s.KA; }
  static __device__ __forceinline__ const double DBM_CONST *KB1(SpC &s) { return s.KB1; }
  static __device__ __forceinline__ const double DBM_CONST *KB2(SpC &s) { return s.KB2; }
  static __device__ __forceinline__ const double DBM_CONST *KE(SpC &s) { return s.KE; }
  static __device__ __forceinline__ const double DBM_CONST *MA(SpC &s) { return s.MA; }
  static __device__ __forceinline__ const double DBM_CONST *MB1(SpC &s) { return s.MB1; }
  static __device__ __forceinline__ const double DBM_CONST *MB2(SpC &s) { return s.MB2; }
  static __device__ __forceinline__ const double DBM_CONST *ME(SpC &s) { return s.ME; }
  static __device__ __forceinline__ double cgx(SpC &s, int g) { return s.cgx[g]; }
  static __device__ __forceinline__ double cgy(SpC &s, int g) { return s.cgy[g]; }
  static __device__ __forceinline__ double omega(SpC &s) { return s.omega; }
};

// Hide a wave-uniform pointer from loop-invariant code motion so that the
// table values it points to are re-read from the scalar cache each row
// instead of being held (and spilled) in scalar registers.
template <typename P> __device__ __forceinline__ P launder(P p) {
#ifndef DBM_NO_LAUNDER
  asm volatile("" : "+s"(p));
#endif
  return p;
}

// The same, and also not before `v` is computed: the table values read
// through the result are loaded where they are used, so that the scalar
// registers hold one block of a table at a time.
// Applied in FP64 only: the FP32 tables fit in scalar registers as they are.
template <typename P, typename V> __device__ __forceinline__ P launder_after(P p, V v) {
#ifndef DBM_NO_LAUNDER
  if constexpr (sizeof(V) == 8) asm volatile("" : "+s"(p) : "v"(v));
#endif
  return p;
}

// DPP whole-wavefront shifts: shr1 gives lane i the value of lane i-1,
// shl1 the value of lane i+1; the lane with no source keeps `old`.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

// Guard-lane variants for the stencil: the lane with no source reads 0
// (bound_ctrl), which lets the compiler fold the move into the consuming
// VALU instruction as a DPP operand.  Only guard lanes see the 0.
__device__ __forceinline__ float shr1(float src) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), kDppWaveShr1, 0xf, 0xf, true));
}
__device__ __forceinline__ float shl1(float src) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), kDppWaveShl1, 0xf, 0xf, true));
}
__device__ __forceinline__ double shr1(double src) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(src), kDppWaveShr1, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(src), kDppWaveShr1, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shl1(double src) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(src), kDppWaveShl1, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(src), kDppWaveShl1, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

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

// Stencil shifts with the edge lane fed from `edge` (a value of the
// neighbouring tile): lane 0 of shr1e and lane 63 of shl1e return `edge`.
__device__ __forceinline__ float shr1e(float src, float edge) { return dpp_shr1(src, edge); }
__device__ __forceinline__ float shl1e(float src, float edge) { return dpp_shl1(src, edge); }
__device__ __forceinline__ double shr1e(double src, double edge) { return dpp_shr1(src, edge); }
__device__ __forceinline__ double shl1e(double src, double edge) { return dpp_shl1(src, edge); }

// Raw buffer access (MUBUF): a 128-bit resource holds the 64-bit base and the
// byte size, the per-lane offset is a VGPR and a wavefront-uniform offset
// (the plane) an SGPR, so a load costs no vector address arithmetic.
// Accesses beyond the size return 0 / are dropped by the hardware.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit data format (gfx9 family)
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           kRsrcWord3);
}
template <typename T> __device__ __forceinline__ T bload(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// Stores of the new distribution: aux bit 1 marks them non-temporal.
constexpr int kStoreAux = DBM_NT_STORE ? 2 : 0;
__device__ __forceinline__ void bstore(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff,
                                        kStoreAux);
}
__device__ __forceinline__ void bstore(rsrc_t r, double v, uint32_t voff, uint32_t soff) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff,
                                        kStoreAux);
}

// Value of lane l (a compile-time constant) broadcast to the wavefront.
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Storage of f.  float (FP32-bulk) and double (FP64) hold each value itself.
// f32x holds each value as its FP32 rounding plus the bfloat16 rounding of
// the remainder (FP32's exponent range, 8 more significant bits: about 32 in
// all, relative error <= 2^-32), in 6 bytes: a buffer of n values is n FP32
// values followed by n 16-bit residuals.  f32x is read and written from FP64
// arithmetic.
// ---------------------------------------------------------------------------
struct f32x {};
template <typename ST> struct Stor;
template <> struct Stor<float> { typedef float C; };
template <> struct Stor<double> { typedef double C; };
template <> struct Stor<f32x> { typedef double C; };
template <typename ST> constexpr bool kSplitStore = std::is_same<ST, f32x>::value;

__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t bf16_round(float x) {  // to nearest, ties to even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ void split_f32x(double v, float &hi, uint16_t &lo) {
  hi = (float)v;
  lo = bf16_round((float)(v - (double)hi));   // v - hi is exact in FP64
}
__device__ __forceinline__ double join_f32x(float hi, uint16_t lo) {
  return (double)hi + (double)bf16_value(lo);
}

// Stochastic rounding of FP32 stores (option of FP32-bulk).  Round-to-nearest
// of f + d, repeated every step on slowly varying fields, makes the rounding
// errors of successive steps alike and lets them add up; rounding up or down
// with probabilities in proportion to the distances makes each store's
// error zero in expectation, so they add up as a random walk instead.
// The random bits are a hash of the cell, the species and the values being
// updated (the state itself): results stay deterministic and do not depend on
// tiling or launch order.
// mix32 is the 32-bit integer finaliser "lowbias32" published by C. Wellons
// (hash-prospector, 2018): xor-shift 16, multiply, xor-shift 15, multiply,
// xor-shift 16, with the two multipliers found there by search.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// f + d rounded to FP32 stochastically with the 8 random bits in the low byte
// of u8: the exact remainder of the nearest sum (exact when |f| >= |d|) plus
// a dither uniform over 256 levels in (-ulp/2, ulp/2), rounded to nearest.
// With E the power of two of sm's exponent (ulp = E 2^-23) the dither is
// E t, t = (u + 1/2) 2^-31 - 2^-24 formed exactly by one multiply-add, and
// er + E t is exact in its multiply-add too.
__device__ __forceinline__ float sr_add(float f, float d, uint32_t u8) {
  const float sm = f + d;
  const float er = d - (sm - f);
  const float E = __uint_as_float(__float_as_uint(sm) & 0x7f800000u);
  const float t = fma((float)(u8 & 0xffu), 0x1p-31f, 0x1p-32f - 0x1p-24f);
  return sm + fma(E, t, er);
}

// Step counter of stochastic rounding: ctr[0] is read by every workgroup at
// the start of a launch; the last workgroup to finish advances it (ctr[1]
// counts the finished workgroups), so each launch draws new random bits.
// No fence is needed: every workgroup's read has returned (its value was
// used) before its increment, the last workgroup writes only after seeing
// all increments, and the next launch sees the write at the kernel boundary.
// (A device-scope fence here would write back every XCD's L2 per workgroup.)
__device__ __forceinline__ void advance_step_counter(uint32_t *ctr, uint32_t step,
                                                     uint32_t nblocks) {
  if (threadIdx.x == 0) {
    const uint32_t done =
        __hip_atomic_fetch_add(&ctr[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == nblocks - 1) {
      __hip_atomic_store(&ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctr[0], step + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The 32-bit key of a row's stochastic roundings: cell, species, launch and
// the values being updated, combined with the golden-ratio multiplier
// 0x9E3779B9 and the odd constants of MurmurHash3's finaliser and xxHash.
__device__ __forceinline__ uint32_t sr_key(uint32_t cell, int s, uint32_t step, const float *v) {
  uint32_t key = cell * 0x9E3779B9u ^ (uint32_t)(s + 1) * 0x85EBCA6Bu ^ step * 0xC2B2AE35u;
#pragma unroll
  for (int i = 0; i < kNV; ++i) key = (key ^ __float_as_uint(v[i])) + (uint32_t)i * 0x27D4EB2Fu;
  return key;
}

// Element access to one buffer of n values (generic kernels).
template <typename ST> struct FV {
  typedef typename Stor<ST>::C C;
  const void *b;
  size_t n;
  __device__ FV(const void *b_, size_t n_) : b(b_), n(n_) {}
  __device__ C operator[](size_t i) const {
    if constexpr (kSplitStore<ST>)
      return join_f32x(((const float *)b)[i], ((const uint16_t *)((const float *)b + n))[i]);
    else
      return ((const ST *)b)[i];
  }
  __device__ void set(size_t i, C v) const {
    if constexpr (kSplitStore<ST>) {
      float hi;
      uint16_t lo;
      split_f32x(v, hi, lo);
      ((float *)b)[i] = hi;
      ((uint16_t *)((float *)b + n))[i] = lo;
    } else {
      ((ST *)b)[i] = (ST)v;
    }
  }
};
// Values of one f buffer (each part, for FP32X): S x 16 planes of I.ps.
__device__ __forceinline__ size_t nvals(const InstDev &I) {
  return (size_t)I.S * kNV * I.ps;
}
template <typename ST> __device__ __forceinline__ FV<ST> fview(const InstDev &I, int b) {
  return FV<ST>(I.buf[b], nvals(I));
}

// One species of one buffer as raw-buffer resources (one-pass kernel):
// value(cell, plane) and store(cell, plane, v); the plane goes to the scalar
// offset.  lane_value takes a per-lane plane (halo loads).
template <typename ST> struct FBuf {
  typedef typename Stor<ST>::C C;
  static constexpr uint32_t es = kSplitStore<ST> ? 4 : sizeof(ST);
  rsrc_t hi, lo;
  uint32_t plb_hi, plb_lo;  // bytes per plane of each part
  __device__ FBuf(const InstDev &I, int b, int s) {
    const size_t plane = I.ps;
    plb_hi = (uint32_t)plane * es;
    plb_lo = (uint32_t)plane * 2u;
    const size_t first = (size_t)s * kNV * plane;
    if constexpr (kSplitStore<ST>) {
      hi = make_rsrc((const float *)I.buf[b] + first, kNV * plb_hi);
      lo = make_rsrc((const uint16_t *)((const float *)I.buf[b] + nvals(I)) + first, kNV * plb_lo);
    } else {
      hi = make_rsrc((const ST *)I.buf[b] + first, kNV * plb_hi);
      lo = hi;
    }
  }
  __device__ C value(uint32_t cell, uint32_t p) const {
    if constexpr (kSplitStore<ST>) {
      const float h = bload<float>(hi, cell * 4u, p * plb_hi);
      const uint16_t l = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(lo, (int)(cell * 2u),
                                                                       (int)(p * plb_lo), 0);
      return join_f32x(h, l);
    } else {
      return bload<ST>(hi, cell * es, p * plb_hi);
    }
  }
  __device__ C lane_value(uint32_t p, uint32_t cell) const {
    if constexpr (kSplitStore<ST>) {
      const float h = bload<float>(hi, p * plb_hi + cell * 4u, 0);
      const uint16_t l = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(lo, (int)(p * plb_lo + cell * 2u), 0, 0);
      return join_f32x(h, l);
    } else {
      return bload<ST>(hi, p * plb_hi + cell * es, 0);
    }
  }
  __device__ void store(uint32_t cell, uint32_t p, C v) const {
    if constexpr (kSplitStore<ST>) {
      float h;
      uint16_t l;
      split_f32x(v, h, l);
      bstore(hi, h, cell * 4u, p * plb_hi);
      __builtin_amdgcn_raw_buffer_store_b16(l, lo, (int)(cell * 2u), (int)(p * plb_lo), kStoreAux);
    } else {
      bstore(hi, v, cell * es, p * plb_hi);
    }
  }
};

// A-block residuals of OM storage (option of FP32-bulk): per species the
// four A-block values also keep the rounding remainder of their FP32 value,
// as a bfloat16 (the encoding of FP32X), in four uint16 planes of stride ps
// that follow the S x 16 FP32 planes of the buffer.
struct AResBuf {
  rsrc_t r;
  uint32_t plb;  // bytes per plane
  __device__ AResBuf(const InstDev &I, int b, int s) {
    plb = (uint32_t)I.ps * 2u;
    r = make_rsrc((const uint16_t *)((const float *)I.buf[b] + nvals(I)) + (size_t)s * 4 * I.ps,
                  4 * plb);
  }
  __device__ uint16_t value(uint32_t cell, uint32_t j) const {
    return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(cell * 2u), (int)(j * plb), 0);
  }
  __device__ void store(uint32_t cell, uint32_t j, uint16_t v) const {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)(cell * 2u), (int)(j * plb), kStoreAux);
  }
};
// The same residuals through plain pointers (conversion kernels), for the
// buffer at `base`.
__device__ __forceinline__ uint16_t *ares_ptr(const InstDev &I, const void *base, int s, int j) {
  return (uint16_t *)((float *)base + nvals(I)) + (size_t)(s * 4 + j) * I.ps;
}

// Lane gather through the LDS crossbar: lane l gets v from lane addr[l] / 4.
__device__ __forceinline__ float bperm(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bperm(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// A value entering the row-to-row state from the prefetch ring.  In FP64 it
// is copied to a register of its own (a copy the compiler cannot fold away):
// otherwise the state keeps the ring slot's registers, the next prefetch
// into that slot lands elsewhere, and the copy back at the loop latch waits
// for it, which drains the prefetch every other row.
__device__ __forceinline__ float carry(float x) { return x; }
__device__ __forceinline__ double carry(double x) {
  double y;
  asm volatile("v_mov_b64 %0, %1" : "=v"(y) : "v"(x));
  return y;
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
  // Reflections about the faces at 0 and n repeat with period 2n.
  int q = r % (2 * n);
  if (q < 0) q += 2 * n;
  flip = q >= n;
  return flip ? 2 * n - 1 - q : q;
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
__device__ __forceinline__ void block_feq(SpC &sp, const T *r, T *f) {
  const T DBM_CONST *KA = launder_after(Tab<T>::KA(sp), r[0]);
  const T DBM_CONST *KE = launder_after(Tab<T>::KE(sp), r[8]);
  const T DBM_CONST *KB1 = launder_after(Tab<T>::KB1(sp), r[4]);
  const T DBM_CONST *KB2 = launder_after(Tab<T>::KB2(sp), r[6]);
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

// Orbit components of one species' 16 values (plane order of Eq.15):
// A = sum, B = alternating sum, X, Y = sums signed by v_x, v_y.
template <typename T>
__device__ __forceinline__ void orbit_parts(const T *c, T *A, T *B, T *X, T *Y) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const T c0 = c[4 * g], c1 = c[4 * g + 1], c2 = c[4 * g + 2], c3 = c[4 * g + 3];
    const T s02 = c0 + c2, s13 = c1 + c3;
    A[g] = s02 + s13;
    B[g] = s02 - s13;
    if ((g & 1) == 0) {
      X[g] = c0 - c2; Y[g] = c1 - c3;
    } else {
      X[g] = (c0 + c3) - (c1 + c2); Y[g] = (c0 + c1) - (c2 + c3);
    }
  }
}

// FP64 raw moments of one species from its orbit sums (see orbit_parts):
// n = sum_g A_g, j = sum_g v_g (X_g, Y_g), E = sum_g q_g A_g.  The sums over
// groups, which feed the temperature's cancellation, are done in FP64.
template <typename T>
__device__ __forceinline__ void species_moments(SpC &sp, const T *A, const T *X, const T *Y,
                                                double &n, double &jx, double &jy, double &E) {
  n = jx = jy = E = 0.0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const double a = (double)A[g];
    n += a;
    jx = fma(sp.vg[g], (double)X[g], jx);
    jy = fma(sp.vg[g], (double)Y[g], jy);
    E = fma(sp.qg[g], a, E);
  }
}

// Per-cell scalar chain in FP64: mixture u and T from the species moments
// (the conservation statement under Eq.6 with Eqs.8-10), then the chemistry
// of Eqs.(1)-(2) within tau (Eq.5): extents xi_r = omega_r tau of the
// mechanism's steps (one common factor keeps every reactant's consumption
// within its density), n^s* = n^s + sum_r a_r^s xi_r, and T* from the energy
// balance with heat Q_r per unit extent.  dn[s] = n^s* - n^s.
struct CellState {
  double ux, uy, Tst, dn[kMaxFusedSpecies];
};

// 1/x: hardware estimate refined by Newton steps (each squares the
// relative error of the estimate): two in FP64 mode (to about an ulp), one in
// FP32-bulk mode, where the result (relative error ~1e-14) only meets
// FP32-rounded quantities.
template <typename T> __device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  if constexpr (sizeof(T) == 8) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// exp(-E_a/(R T)): FP64 in FP64 mode; in FP32-bulk mode the rate only sets a
// source that is itself rounded to FP32, so it is evaluated in FP32.
template <typename T> __device__ __forceinline__ double arrhenius(double x);
template <> __device__ __forceinline__ double arrhenius<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ double arrhenius<float>(double x) {
  return (double)__expf((float)x);
}

// `mom(q, s)` returns moment q (n, j_x, j_y, E) of species s at this lane's
// cell.
template <typename T, int S, typename Mom>
__device__ __forceinline__ void cell_chain(const InstDev &I, SpC *sp, Mom mom, CellState &cs) {
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double n = mom(0, s);
    rho = fma(sp[s].m, n, rho);
    px = fma(sp[s].m, mom(1, s), px);
    py = fma(sp[s].m, mom(2, s), py);
    e = fma(sp[s].m, mom(3, s), e);
    kn = fma(sp[s].K, n, kn);
  }
  const double irho = recip<T>(rho);
  cs.ux = px * irho;
  cs.uy = py * irho;
  const double ikn = recip<T>(kn);
  const double Tm = (e - rho * (cs.ux * cs.ux + cs.uy * cs.uy)) * ikn;
  cs.Tst = Tm;
#pragma unroll
  for (int s = 0; s < S; ++s) cs.dn[s] = 0.0;
  const int nr = I.nreact;
  if (nr > 0) {
    // Everything below is linear in the extents, so the unscaled sums are
    // accumulated step by step and the common clamp factor (needed only when
    // some reactant would be overdrawn) multiplies them at the end.
    const double iT = recip<T>(Tm);
    double use[S], sdk = 0.0, heat = 0.0, dn[S];
#pragma unroll
    for (int s = 0; s < S; ++s) use[s] = dn[s] = 0.0;
#pragma unroll 1
    for (int r = 0; r < nr; ++r) {
      const double nF = fmax(mom(0, I.rfuel[r]), 0.0);
      const double nO = fmax(mom(0, I.roxid[r]), 0.0);
      const double x = I.rk[r] * nF * nO * arrhenius<T>(-I.rEa[r] * iT) * sp[0].tau;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        use[s] = fma(I.rneg[r][s], x, use[s]);
        dn[s] = fma(I.ra[r][s], x, dn[s]);
      }
      sdk = fma(I.rdK[r], x, sdk);
      heat = fma(I.rQ2[r], x, heat);
    }
    bool over = false;
#pragma unroll
    for (int s = 0; s < S; ++s) over = over || use[s] > fmax(mom(0, s), 0.0);
    if (over) {
      double scale = 1.0;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const double avail = fmax(mom(0, s), 0.0);
        if (use[s] > avail) scale = fmin(scale, avail * recip<T>(use[s]));
      }
      sdk *= scale;
      heat *= scale;
#pragma unroll
      for (int s = 0; s < S; ++s) dn[s] *= scale;
    }
    // sum (D+I) n* T* = sum (D+I) n T + 2 sum_r Q_r xi_r
    cs.Tst = fma(Tm, kn, heat) * recip<T>(kn + sdk);
#pragma unroll
    for (int s = 0; s < S; ++s) cs.dn[s] = dn[s];
  }
}

// block_feq restricted to the axis group g0 (0 or 2) and the diagonal group
// g0 + 1: the eight values of planes 4 g0 .. 4 g0 + 7.
template <typename T>
__device__ __forceinline__ void block_feq_pair(SpC &sp, const T *r, int g0, T *f) {
  const T DBM_CONST *KA = launder_after(Tab<T>::KA(sp), r[0]);
  const T DBM_CONST *KE = launder_after(Tab<T>::KE(sp), r[8]);
  const T DBM_CONST *KB1 = launder_after(Tab<T>::KB1(sp), r[4]);
  const T DBM_CONST *KB2 = launder_after(Tab<T>::KB2(sp), r[6]);
#pragma unroll
  for (int lg = 0; lg < 2; ++lg) {
    const int g = g0 + lg;
    T al = KA[g * 4] * r[0], xi = KE[g * 4] * r[8], ps = KE[g * 4] * r[12];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      al = fma(KA[g * 4 + j], r[j], al);
      xi = fma(KE[g * 4 + j], r[8 + j], xi);
      ps = fma(KE[g * 4 + j], r[12 + j], ps);
    }
    T *o = f + 4 * lg;
    if (lg == 0) {  // axis group: B from the (v_x^2 - v_y^2) rows
      const T be = fma(KB1[g0 + 1], r[5], KB1[g0] * r[4]);
      const T p = al + be, m = al - be;
      o[0] = p + xi; o[1] = m + ps; o[2] = p - xi; o[3] = m - ps;
    } else {        // diagonal group: B from the v_x v_y rows
      const T be = fma(KB2[g0 + 1], r[7], KB2[g0] * r[6]);
      const T p = al + be, m = al - be;
      const T sm = xi + ps, df = xi - ps;
      o[0] = p + sm; o[1] = m - df; o[2] = p - sm; o[3] = m + df;
    }
  }
}

// Collision + reaction + force of one species in moment space:
//   df = f^eq(n*, u, T*) + [f^eq(n, u+, T+) - f^eq(n, u^s, T^s)] - f
//      = M^{-1} (g - M f)
// with g the combined equilibrium moments.  The rows of g - M f that carry
// mass, momentum and energy are differenced in FP64 from the FP64 moments,
// so the update conserves them to the rounding of the (small) difference
// itself; the other rows are differenced in the storage precision.
template <typename T>
__device__ __forceinline__ void collision_rhs(const InstDev &I, SpC &sp, const T *A,
                                              const T *B, const T *X, const T *Y, double n,
                                              double jx, double jy, double E, double ns,
                                              double ux, double uy, double Tst, T *d) {
  const double K = sp.K, th = Tst * sp.inv_m, u2 = ux * ux + uy * uy;
  T r[16];
  eq_rhs<T>((T)ns, (T)ux, (T)uy, (T)th, (T)K, r);
  double d0 = ns - n, d1 = ns * fma(K, th, u2) - E, d8 = ns * ux - jx, d12 = ns * uy - jy;
  const bool force = I.force && n > 1e-300;
  double fd[16];
  if (force) {
    const double inv_n = recip<T>(n);
    const double us = jx * inv_n, vs = jy * inv_n;
    const double Ts = sp.m * (E * inv_n - us * us - vs * vs) * sp.inv_K;
    double Td = Ts;
    if (I.fmode == DBM_FORCE_T_EXACT)
      Td = Ts - sp.m * sp.tau * sp.tau * (I.ax * I.ax + I.ay * I.ay) * sp.inv_K;
    double r1[16], r2[16];
    eq_rhs<double>(n, us + sp.tau * I.ax, vs + sp.tau * I.ay, Td * sp.inv_m, K, r1);
    eq_rhs<double>(n, us, vs, Ts * sp.inv_m, K, r2);
#pragma unroll
    for (int k = 0; k < 16; ++k) fd[k] = r1[k] - r2[k];
    d0 += fd[0];
    d1 += fd[1];
    d8 += fd[8];
    d12 += fd[12];
  }
  const T DBM_CONST *MA = launder_after(Tab<T>::MA(sp), r[2]);
  const T DBM_CONST *MB1 = launder_after(Tab<T>::MB1(sp), r[4]);
  const T DBM_CONST *MB2 = launder_after(Tab<T>::MB2(sp), r[6]);
  const T DBM_CONST *ME = launder_after(Tab<T>::ME(sp), r[9]);
  d[0] = (T)d0;
  d[1] = (T)d1;
  d[8] = (T)d8;
  d[12] = (T)d12;
#pragma unroll
  for (int row = 2; row < 4; ++row) {
    T m = MA[row * 4] * A[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) m = fma(MA[row * 4 + j], A[j], m);
    d[row] = r[row] - m;
  }
  d[4] = r[4] - fma(MB1[1], B[2], MB1[0] * B[0]);
  d[5] = r[5] - fma(MB1[3], B[2], MB1[2] * B[0]);
  d[6] = r[6] - fma(MB2[1], B[3], MB2[0] * B[1]);
  d[7] = r[7] - fma(MB2[3], B[3], MB2[2] * B[1]);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    T mx = ME[row * 4] * X[0], my = ME[row * 4] * Y[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      mx = fma(ME[row * 4 + j], X[j], mx);
      my = fma(ME[row * 4 + j], Y[j], my);
    }
    d[8 + row] = r[8 + row] - mx;
    d[12 + row] = r[12 + row] - my;
  }
  if (force) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k != 0 && k != 1 && k != 8 && k != 12) d[k] += (T)fd[k];
  }
}

template <typename T>
__device__ __forceinline__ void collision_delta(const InstDev &I, SpC &sp, const T *A,
                                                const T *B, const T *X, const T *Y, double n,
                                                double jx, double jy, double E, double ns,
                                                double ux, double uy, double Tst, T *df) {
  T d[16];
  collision_rhs<T>(I, sp, A, B, X, Y, n, jx, jy, E, ns, ux, uy, Tst, d);
  block_feq<T>(sp, d, df);
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
// Rows of loads kept in flight per wavefront.
#ifndef DBM_PREFETCH
#define DBM_PREFETCH 2
#endif
constexpr int kPrefetch = DBM_PREFETCH;
static_assert(kPrefetch >= 2, "the prefetch ring needs two or more slots");
// Rows of loads in flight per wavefront in the one-pass kernel: three for the
// four-species FP32 Euler form (1% faster on the 4096^2 and 2048^2 shear
// layers than two), kPrefetch elsewhere (three slowed the Runge-Kutta and
// stochastic-rounding forms by 7-11% through register pressure).
template <typename ST, int S, bool RKC, bool PIPE, bool SR, bool CW>
constexpr int kRing = (std::is_same<ST, float>::value && S == 4 && !RKC && !PIPE && !SR && !CW)
                          ? (kPrefetch > 3 ? kPrefetch : 3)
                          : kPrefetch;

// The 12 planes with a nonzero v_x, in plane order, and the halo columns each
// needs: x0-1 and x0+64 always, and x0-2 (v_x > 0) or x0+65 (v_x < 0).
__host__ __device__ constexpr int xplane(int j) {
  return j < 2 ? 2 * j : (j < 6 ? j + 2 : (j < 8 ? 2 * j - 4 : j + 4));
}
__host__ __device__ constexpr int xplane_index(int i) {
  return i < 4 ? i / 2 : (i < 8 ? i - 2 : (i < 12 ? i / 2 + 2 : i - 4));
}
static_assert(xplane(0) == 0 && xplane(1) == 2 && xplane(5) == 7 && xplane(7) == 10 &&
                  xplane(8) == 12 && xplane(11) == 15 && xplane_index(10) == 7 &&
                  xplane_index(13) == 9 && plane_sx(10) != 0 && plane_sx(9) == 0 && plane_sx(1) == 0,
              "x-moving planes of the D2V16 ordering");
constexpr int kXPlanes = 12;
constexpr int kHaloLanes = 3 * kXPlanes;

// Chain wavefront (CW, S <= 3): the workgroup has one more wavefront,
// which forms the mixture chain (u, T, reaction extents, T*) of row k+1
// from the species' moments while the species wavefronts form row k's
// collision and stencils, and publishes it through LDS (u_x, u_y, T*, dn^s
// per cell).  One barrier per row, as without it: the species publish row
// k+1's moments (from the prefetched values) and find row k's chain formed
// during row k-1.  The species wavefronts shed the FP64 chain and with
// S = 3 the fourth SIMD of a CU gets work.
template <int S, bool CW> constexpr int kChainRows = CW ? 3 + S : 1;

// Rows a tile's row loop runs: FP64 arithmetic runs whole ring cycles,
// computing (not storing) up to kPrefetch-1 rows past the tile (kSteady in
// fused_tile); the chain wavefront runs the same number of row barriers.
template <typename T> constexpr bool kSteadyRows = sizeof(T) == 8;
__device__ __forceinline__ int rows_run(bool steady, int rows) {
  return steady ? (rows + kPrefetch - 1) / kPrefetch * kPrefetch : rows;
}

// Software pipeline over rows (PIPE, FP32): row k+1's moments, mixture
// chain and collision are formed while row k's stencils are (their inputs
// are already in registers: the prefetched row and the carried y-state),
// which gives the scheduler two independent streams of work per row.  It
// shortens each wavefront's rows (small, latency-bound grids gain) at 16
// more VGPRs (large, throughput-bound grids lose); the tuner picks.

// FP32 chain-wavefront rows form their stencils before the row barrier (in
// FP64 the extra live values would not fit in registers).
#ifndef DBM_EARLY_STENCIL
#define DBM_EARLY_STENCIL 1
#endif
// Halo distribution: LDS crossbar gather (1) or lane reads (0), per type.
#ifndef DBM_GATHER_F32
#define DBM_GATHER_F32 1
#endif
#ifndef DBM_GATHER_F64
#define DBM_GATHER_F64 1
#endif
template <typename T> constexpr bool kHaloGather = sizeof(T) == 4 ? DBM_GATHER_F32 : DBM_GATHER_F64;

// One wavefront's share of a tile: species `s`, 64 lanes = columns
// x0 .. x0+63, rows y0 .. y0+rows-1.  `mom` is the workgroup's LDS
// exchange of per-cell FP64 moments, double-buffered by row parity.
template <typename ST, int S, int LIM, bool RKC, bool PIPE, bool SR, bool CW>
__device__ __forceinline__ void fused_tile(const InstDev &I, const int s, int x0, int y0,
                                           int rows, int in_idx, int fn_idx, int out_idx,
                                           typename Stor<ST>::C alpha, uint32_t step,
                                           double (*mom)[4 * S][kWave],
                                           double (*chn)[kChainRows<S, CW>][kWave]) {
  typedef typename Stor<ST>::C T;                  // arithmetic type
  constexpr int kPf = kRing<ST, S, RKC, PIPE, SR, CW>;   // rows of loads in flight
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = I.nx, ny = I.ny, bcy = I.bcy;
  // One set of buffer resources per species and buffer (its 16 planes,
  // under 4 GiB by a host check); offsets below them are 32-bit byte counts:
  // the plane in the SGPR offset, the cell in the VGPR offset.
  const FBuf<ST> bin(I, in_idx, s), bfn(I, fn_idx, s), bout(I, out_idx, s);
  const int col = x0 + lane;                       // column held by this lane
  const int lcol = map_x(col, nx, I.bcx);          // where its value lives
  const bool writer = col < nx;
  const int yend = y0 + rows;

  auto load = [&](int i, int roff, bool flip) -> T {
    const uint32_t p = flip ? mirror_y(i) : i;
    return bin.value((uint32_t)(roff + lcol), p);
  };
  // Compact halo: lane 3j+w (j < 12) holds plane xplane(j) at column x0-1
  // (w = 0), x0-2 or x0+65 (w = 1, by the sign of v_x), x0+64 (w = 2).
  // Lanes 36..63 re-read lane 0's value (in bounds, never used).
  uint32_t hplane, hcol;
  {
    const int hl = lane < kHaloLanes ? lane : 0;
    const int j = hl / 3, w = hl - 3 * j;
    const int hp = xplane(j);
    const int hc = w == 0 ? x0 - 1 : (w == 2 ? x0 + kWave : (plane_sx(hp) > 0 ? x0 - 2 : x0 + kWave + 1));
    hplane = (uint32_t)hp;
    hcol = (uint32_t)map_x(hc, nx, I.bcx);
  }
  // Gather addresses of the halo: h1 puts slot 0 (x0-1) in lane 0 and slot 2
  // (x0+64) in lane 63; h2 broadcasts slot 1.  Plane j adds 12 j bytes.
  const int hidx1 = lane == kWave - 1 ? 8 : 0;

  // State carried between rows, per plane i:
  //   c  = f at the current row k
  //   y1 = f_k - f_{k-1}           (v_y > 0)   or f_{k+1}   (v_y < 0)
  //   y2 = slope at row k-1        (v_y > 0)   or slope at row k (v_y < 0)
  // Row y0 is loaded first (the first collision needs only it), then the
  // other rows of the stencil: y0-2, y0-1 (v_y > 0) or y0-1, y0+1 (v_y < 0).
  T c[kNV], y1[kNV], y2[kNV], pa[kNV], pb[kNV];
  {
    bool fm2, fm1, f0, fp1;
    const int rm2 = map_y(y0 - 2, ny, bcy, fm2) * nx, rm1 = map_y(y0 - 1, ny, bcy, fm1) * nx;
    const int r0 = map_y(y0, ny, bcy, f0) * nx, rp1 = map_y(y0 + 1, ny, bcy, fp1) * nx;
#pragma unroll
    for (int i = 0; i < kNV; ++i) c[i] = load(i, r0, f0);
#pragma unroll
    for (int i = 0; i < kNV; ++i) {
      const int sy = plane_sy(i);
      if (sy > 0) {
        pa[i] = load(i, rm2, fm2);
        pb[i] = load(i, rm1, fm1);
      } else if (sy < 0) {
        pa[i] = load(i, rm1, fm1);
        pb[i] = load(i, rp1, fp1);
      }
    }
  }
  auto start_state = [&]() {
#pragma unroll
    for (int i = 0; i < kNV; ++i) {
      const int sy = plane_sy(i);
      if (sy > 0) {
        y1[i] = c[i] - pb[i];
        y2[i] = slope_pos<LIM>(pb[i] - pa[i], c[i] - pb[i]);
      } else if (sy < 0) {
        y1[i] = pb[i];
        y2[i] = slope_neg<LIM>(c[i] - pa[i], pb[i] - c[i]);
      } else {
        y1[i] = T(0);
        y2[i] = T(0);
      }
    }
  };

  // New values consumed by row k: row k+1 (v_y >= 0) or k+2 (v_y < 0), and
  // the x-halo of row k itself (an interior row: no y mapping).
  auto issue = [&](int k, T *dst, T &halo) {
    bool fa, fb;
    const int ra = map_y(k + 1, ny, bcy, fa) * nx, rb = map_y(k + 2, ny, bcy, fb) * nx;
#pragma unroll
    for (int i = 0; i < kNV; ++i) dst[i] = plane_sy(i) < 0 ? load(i, rb, fb) : load(i, ra, fa);
    halo = bin.lane_value(hplane, hcol + (uint32_t)(k * nx));
  };

  // Collision of row k from its values fr: own FP64 moments to LDS, one
  // barrier, the mixture chain from every species' moments, then the
  // moment-space collision into dfo.
  auto collide = [&](int k, const T *fr, SpC *sp, SpC &me, T *dfo) {
    T oA[4], oB[4], oX[4], oY[4];
    orbit_parts<T>(fr, oA, oB, oX, oY);
    double n0, jx0, jy0, E0;
    species_moments<T>(me, oA, oX, oY, n0, jx0, jy0, E0);
    double(*mb)[kWave] = mom[k & 1];
    mb[0 * S + s][lane] = n0;
    mb[1 * S + s][lane] = jx0;
    mb[2 * S + s][lane] = jy0;
    mb[3 * S + s][lane] = E0;
    __syncthreads();
    CellState cs;
    cell_chain<T, S>(I, sp, [&](int q, int sp_) { return mb[q * S + sp_][lane]; }, cs);
    double dn_own = cs.dn[0];
#pragma unroll
    for (int q = 1; q < S; ++q)
      if (q == s) dn_own = cs.dn[q];   // wave-uniform select, no indexed array
    collision_delta<T>(I, me, oA, oB, oX, oY, n0, jx0, jy0, E0, n0 + dn_own, cs.ux, cs.uy,
                       cs.Tst, dfo);
  };
  // Chain wavefront: this species' FP64 moments of row k (values fr) to LDS.
  auto publish = [&](int k, const T *fr, SpC &me) {
    T oA[4], oB[4], oX[4], oY[4];
    orbit_parts<T>(fr, oA, oB, oX, oY);
    double n0, jx0, jy0, E0;
    species_moments<T>(me, oA, oX, oY, n0, jx0, jy0, E0);
    double(*mb)[kWave] = mom[k & 1];
    mb[0 * S + s][lane] = n0;
    mb[1 * S + s][lane] = jx0;
    mb[2 * S + s][lane] = jy0;
    mb[3 * S + s][lane] = E0;
  };
  // Row k consumes ring slot d and refills the slot freed by row k-1 with the
  // values of row k+D-1, so D rows of loads are in flight.  (Issuing the
  // first slots before the first collision measured slower than after it.)
  T ring[kPf][kNV];
  T hring[kPf];
  constexpr bool kPipe = PIPE && sizeof(T) == 4;
  constexpr bool kCW = CW;
  static_assert(!(kPipe && kCW), "the chain wavefront replaces the row pipeline");
  T df[kNV];
  if constexpr (kPipe) {   // needs row y0 only: overlaps the other rows' loads
    SpC *sp = launder(as_const(I.sp));
    collide(y0, c, sp, sp[s], df);
  }
  if constexpr (kCW) {     // row y0's moments for the chain wavefront's first chain
    SpC *sp = launder(as_const(I.sp));
    publish(y0, c, sp[s]);
    __syncthreads();
  }
  start_state();
#pragma unroll
  for (int d = 0; d < kPf - 1; ++d)
    if (y0 + d < yend) issue(y0 + d, ring[d], hring[d]);

  // kSteady (FP64 arithmetic): the loop body has no conditional loads or
  // rows, so the compiler's wait counts stay exact across the loop latch
  // (with them it waits for every load in flight there).  Rows past the
  // tile's end are then computed (from in-range rows: map_y wraps, clamps
  // or mirrors every index) but not stored.  In FP32 the conditional form
  // measured faster.
  constexpr bool kSteady = kSteadyRows<T>;
  auto row = [&](int k, const T *cur, const T hcur, T *refill, T &hrefill) {
    if (kSteady || k + kPf - 1 < yend) issue(k + kPf - 1, refill, hrefill);
    const int rk = k * nx;
    const int rkn = k < ny ? rk : (ny - 1) * nx;   // f^n row (a row past the grid: not stored)
    SpC *sp = launder(as_const(I.sp));
    SpC &me = sp[s];
    // Halo of the x-moving planes and the advection coefficients, fetched
    // first so that their latency hides behind the moment exchange: h1 =
    // f(x0-1) in lane 0 and f(x0+64) in lane 63; h2 = f(x0-2) (v_x > 0) or
    // f(x0+65) (v_x < 0).
    // (FP32 only: in FP64 the 24 extra doubles would not fit in registers,
    // so there each plane gathers its halo where it is used.)
    auto halo = [&](int j, T &a, T &b) {
      if constexpr (kHaloGather<T>) {
        a = bperm(hidx1 + 12 * j, hcur);
        b = bperm(4 + 12 * j, hcur);
      } else {
        a = lane == 0 ? readlane(hcur, 3 * j) : readlane(hcur, 3 * j + 2);
        b = readlane(hcur, 3 * j + 1);
      }
    };
    constexpr bool kEarlyHalo = sizeof(T) == 4;
    T h1[kXPlanes], h2[kXPlanes];
    if constexpr (kEarlyHalo) {
#pragma unroll
      for (int j = 0; j < kXPlanes; ++j) halo(j, h1[j], h2[j]);
    }
    T cgx[4], cgy[4];
    if constexpr (kEarlyHalo) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        cgx[g] = Tab<T>::cgx(me, g);
        cgy[g] = Tab<T>::cgy(me, g);
      }
    }
    // Row k's collision: from the previous row (pipelined) or here.  With a
    // chain wavefront: publish row k+1's moments, one barrier, then row k's
    // collision from the chain the chain wavefront formed during row k-1.
    if constexpr (!kPipe && !kCW) collide(k, c, sp, me, df);
    // Chain wavefront, stencil first (kEarlyStencil): the stencils of row k
    // and the carried rows' update are formed before the row's barrier, so
    // they overlap the wait for the chain; the collision and the combine
    // follow it.
    constexpr bool kEarlyStencil = kCW && DBM_EARLY_STENCIL && sizeof(T) == 4;
    // Row k's collision from the chain and moments in LDS, and the
    // publication of row k+1's moments (from its values fn1) before it.
    auto cw_collide = [&](const T *fn1, const T *oA, const T *oB, const T *oX, const T *oY) {
      if (k + 1 < yend) publish(k + 1, fn1, me);
      __syncthreads();
      double(*cb)[kWave] = chn[k & 1];
      const double ux = cb[0][lane], uy = cb[1][lane], Tst = cb[2][lane];
      const double dn = cb[3 + s][lane];
      // Row k's own moments are the ones this wavefront published for the
      // chain (from the same values); only this wavefront writes its slots.
      double(*mk)[kWave] = mom[k & 1];
      const double n0 = mk[0 * S + s][lane], jx0 = mk[1 * S + s][lane];
      const double jy0 = mk[2 * S + s][lane], E0 = mk[3 * S + s][lane];
      collision_delta<T>(I, me, oA, oB, oX, oY, n0, jx0, jy0, E0, n0 + dn, ux, uy, Tst, df);
    };
    if constexpr (kCW && !kEarlyStencil) {
      if (k + 1 < yend) {
        T fn1[kNV];
#pragma unroll
        for (int i = 0; i < kNV; ++i) fn1[i] = plane_sy(i) < 0 ? y1[i] : cur[i];
        publish(k + 1, fn1, me);
      }
      __syncthreads();
      double(*cb)[kWave] = chn[k & 1];
      const double ux = cb[0][lane], uy = cb[1][lane], Tst = cb[2][lane];
      const double dn = cb[3 + s][lane];
      // Row k's own moments are the ones this wavefront published for the
      // chain (from the same values); only this wavefront writes its slots.
      double(*mk)[kWave] = mom[k & 1];
      const double n0 = mk[0 * S + s][lane], jx0 = mk[1 * S + s][lane];
      const double jy0 = mk[2 * S + s][lane], E0 = mk[3 * S + s][lane];
      T oA[4], oB[4], oX[4], oY[4];
      orbit_parts<T>(c, oA, oB, oX, oY);
      collision_delta<T>(I, me, oA, oB, oX, oY, n0, jx0, jy0, E0, n0 + dn, ux, uy, Tst, df);
    }
    // Pipelined: row k+1's values are the prefetched row (v_y >= 0) or the
    // carried next value (v_y < 0); form its collision now.
    T dfn[kNV];
    if constexpr (kPipe) {
      if (k + 1 < yend) {
        T fn1[kNV];
#pragma unroll
        for (int i = 0; i < kNV; ++i) fn1[i] = plane_sy(i) < 0 ? y1[i] : cur[i];
        collide(k + 1, fn1, sp, me, dfn);
      }
    }
    // f^n of the Runge-Kutta combine
    T fnv[kNV];
    if constexpr (RKC) {
#pragma unroll
      for (int i = 0; i < kNV; ++i) fnv[i] = bfn.value((uint32_t)(rkn + lcol), i);
    }
    const T om = Tab<T>::omega(me);
    T res[kNV];
    // Stochastic rounding: the increment d is formed apart from f and the
    // sum rounded once, with 8 random bits per value from four independent
    // hashes per lane and row of one key (cell, species, launch, state).
    constexpr bool kSR = SR && std::is_same<ST, float>::value;
    uint32_t rb[4];
    if constexpr (kSR) {
      const uint32_t key = sr_key((uint32_t)(rk + col), s, step, c);
      rb[0] = mix32(key);
      rb[1] = mix32(key ^ 0x68E31DA4u);
      rb[2] = mix32(key ^ 0xB5297A4Du);
      rb[3] = mix32(key ^ 0x1B56C4E9u);
    }
    auto finish = [&](int i, T a, T f) {
      if constexpr (kSR) {
        T d = fma(om, df[i], a);
        if constexpr (RKC) d = fma(alpha, (fnv[i] - f) - d, d);
        res[i] = sr_add(f, d, rb[i >> 2] >> (8 * (i & 3)));
      } else {
        res[i] = fma(om, df[i], a);
        // alpha + beta = 1 in every stage: res + alpha (f^n - res) rounds
        // only the (small) stage difference
        if constexpr (RKC) res[i] = fma(alpha, fnv[i] - res[i], res[i]);
      }
      if constexpr (!kEarlyHalo)
        if (writer && (!kSteady || k < yend)) bout.store((uint32_t)(rk + col), i, res[i]);
    };
    // Plane i: f (out) and its value plus advection increment (with
    // stochastic rounding the increment alone); advances the carried rows.
    auto advect = [&](int i, T &f) -> T {
      const int g = i >> 2, sx = plane_sx(i), sy = plane_sy(i);
      f = c[i];
      T a = kSR ? T(0) : f;
      // x: NND difference from adjacent lanes.
      // Differences and limited slopes of the neighbouring lanes are the
      // same quantities one lane over, so each is formed once and shifted.
      // The edge lanes take the tile's halo.
      if (sx != 0) {
        const int j = xplane_index(i);
        if constexpr (!kEarlyHalo) halo(j, h1[j], h2[j]);
        // Each edge operand is formed before its last use as a shift's
        // `old` value, so the shifts can write in place.
        const T dl = f - h1[j];                      // lane 0: f_{x0} - f_{x0-1}
        const T e = sx > 0 ? h1[j] - h2[j] : h2[j] - h1[j];
        const T dp = shl1e(f, h1[j]) - f;            // f_{j+1} - f_j
        T Dx;
        if (sx > 0) {
          const T sle = slope_pos<LIM>(e, dl);       // lane 0: slope at x0-1
          const T d0 = shr1e(dp, dl);                // f_j - f_{j-1}
          const T sl = slope_pos<LIM>(d0, dp);       // limited slope at j
          Dx = fma(T(0.5), sl - shr1e(sl, sle), d0);
        } else {
          const T sle = slope_neg<LIM>(dl, dp);      // lane 0: slope at x0
          const T dhi = shl1e(dp, e);                // lane 63: f_{x0+65} - f_{x0+64}
          const T sl = slope_neg<LIM>(dp, dhi);      // limited slope at j+1
          Dx = fma(T(-0.5), sl - shr1e(sl, sle), dp);
        }
        const T cx = kEarlyHalo ? cgx[g] : Tab<T>::cgx(me, g);
        a = (sx > 0) ? fma(-cx, Dx, a) : fma(cx, Dx, a);
      }
      // y: NND difference from the carried rows; advance the state.
      const T fnew = cur[i];
      if (sy > 0) {
        const T dn = fnew - f;
        const T sk = slope_pos<LIM>(y1[i], dn);
        const T Dy = y1[i] + T(0.5) * (sk - y2[i]);
        a = fma(-(kEarlyHalo ? cgy[g] : Tab<T>::cgy(me, g)), Dy, a);
        c[i] = carry(fnew);
        y1[i] = dn;
        y2[i] = sk;
      } else if (sy < 0) {
        const T n1 = y1[i];
        const T dlo = n1 - f, dhi = fnew - n1;
        const T tk1 = slope_neg<LIM>(dlo, dhi);
        const T Dy = dlo - T(0.5) * (tk1 - y2[i]);
        a = fma(kEarlyHalo ? cgy[g] : Tab<T>::cgy(me, g), Dy, a);
        c[i] = n1;
        y1[i] = carry(fnew);
        y2[i] = tk1;
      } else {
        c[i] = carry(fnew);
      }
      return a;
    };
    if constexpr (kEarlyStencil) {
      T oA[4], oB[4], oX[4], oY[4];
      orbit_parts<T>(c, oA, oB, oX, oY);
      T acc[kNV], fk[kNV];
#pragma unroll
      for (int i = 0; i < kNV; ++i) acc[i] = advect(i, fk[i]);
      cw_collide(c, oA, oB, oX, oY);   // c now holds row k+1's values
#pragma unroll
      for (int i = 0; i < kNV; ++i) finish(i, acc[i], fk[i]);
    } else {
#pragma unroll
      for (int i = 0; i < kNV; ++i) {
        T f;
        const T a = advect(i, f);
        finish(i, a, f);
      }
    }
    // FP32: one masked block of stores per row (lanes past nx hold wrapped
    // or clamped copies and write nothing), so that the row is one basic
    // block for the scheduler.
    if constexpr (kEarlyHalo) {
      if (writer) {
#pragma unroll
        for (int i = 0; i < kNV; ++i) bout.store((uint32_t)(rk + col), i, res[i]);
      }
    }
    if constexpr (kPipe) {
#pragma unroll
      for (int i = 0; i < kNV; ++i) df[i] = dfn[i];
    }
  };

  for (int k = y0; k < yend; k += kPf) {
#pragma unroll
    for (int d = 0; d < kPf; ++d) {
      if (kSteady || k + d < yend)
        row(k + d, ring[d], hring[d], ring[(d + kPf - 1) % kPf],
            hring[(d + kPf - 1) % kPf]);
    }
  }
}

// Split form of the one-pass stage, for grids too small to fill the chip:
// each species is carried by two wavefronts, half h holding the planes of
// groups 2h and 2h+1 (planes 8h .. 8h+7: one axis group and one diagonal
// group, so both halves have the same plane types and run the same code).
// Per row each half publishes its orbit parts and partial FP64 moments
// through LDS; after the row's barrier both halves form the species' full
// moments, the mixture chain and the moment-space collision, and each
// updates its own eight planes.  Twice the wavefronts at about two thirds of
// the work each.
constexpr int kHalfPlanes = 8;
constexpr int kHalfXPlanes = 6;                     // local planes 0, 2, 4..7
constexpr int kHalfHaloLanes = 3 * kHalfXPlanes;

template <typename T, int S, int LIM, bool RKC>
__device__ __forceinline__ void fused_tile_split(const InstDev &I, const int s, const int h,
                                                 int x0, int y0, int rows, int in_idx,
                                                 int fn_idx, int out_idx, T alpha,
                                                 T (*orb)[S][16][kWave],
                                                 double (*pm)[4][S][2][kWave]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = I.nx, ny = I.ny, bcy = I.bcy;
  constexpr uint32_t es = sizeof(T);
  const size_t plane = I.ps;
  const uint32_t plb = (uint32_t)plane * es;       // bytes per plane
  const uint32_t spb = kNV * plb;                  // bytes per species
  const rsrc_t rin = make_rsrc((const T *)I.buf[in_idx] + (size_t)s * kNV * plane, spb);
  const rsrc_t rfn = make_rsrc((const T *)I.buf[fn_idx] + (size_t)s * kNV * plane, spb);
  const rsrc_t rout = make_rsrc((const T *)I.buf[out_idx] + (size_t)s * kNV * plane, spb);
  const uint32_t pob = (uint32_t)(kHalfPlanes * h) * plb;   // this half's first plane
  const int col = x0 + lane;
  const int lcol = map_x(col, nx, I.bcx);
  const bool writer = col < nx;
  const int yend = y0 + rows;

  // Local plane j is plane 8h + j; its y-mirror stays in its group.
  auto load = [&](int j, int roff, bool flip) -> T {
    const uint32_t p = flip ? mirror_y(j) : j;
    return bload<T>(rin, (uint32_t)(roff + lcol) * es, pob + p * plb);
  };
  // Compact halo of the six x-moving planes, as in the full form.
  uint32_t hoff;
  {
    const int hl = lane < kHalfHaloLanes ? lane : 0;
    const int j = hl / 3, w = hl - 3 * j;
    const int hp = xplane(j);
    const int hcol = w == 0 ? x0 - 1 : (w == 2 ? x0 + kWave : (plane_sx(hp) > 0 ? x0 - 2 : x0 + kWave + 1));
    hoff = pob + (uint32_t)hp * plb + (uint32_t)map_x(hcol, nx, I.bcx) * es;
  }
  const int hidx1 = lane == kWave - 1 ? 8 : 0;

  T c[kHalfPlanes], y1[kHalfPlanes], y2[kHalfPlanes];
  {
    bool fm2, fm1, f0, fp1;
    const int rm2 = map_y(y0 - 2, ny, bcy, fm2) * nx, rm1 = map_y(y0 - 1, ny, bcy, fm1) * nx;
    const int r0 = map_y(y0, ny, bcy, f0) * nx, rp1 = map_y(y0 + 1, ny, bcy, fp1) * nx;
#pragma unroll
    for (int j = 0; j < kHalfPlanes; ++j) {
      const int sy = plane_sy(j);
      if (sy > 0) {
        const T a = load(j, rm2, fm2), b = load(j, rm1, fm1), cc = load(j, r0, f0);
        c[j] = cc;
        y1[j] = cc - b;
        y2[j] = slope_pos<LIM>(b - a, cc - b);
      } else if (sy < 0) {
        const T a = load(j, rm1, fm1), cc = load(j, r0, f0), n1 = load(j, rp1, fp1);
        c[j] = cc;
        y1[j] = n1;
        y2[j] = slope_neg<LIM>(cc - a, n1 - cc);
      } else {
        c[j] = load(j, r0, f0);
        y1[j] = T(0);
        y2[j] = T(0);
      }
    }
  }
  auto issue = [&](int k, T *dst, T &halo) {
    bool fa, fb;
    const int ra = map_y(k + 1, ny, bcy, fa) * nx, rb = map_y(k + 2, ny, bcy, fb) * nx;
#pragma unroll
    for (int j = 0; j < kHalfPlanes; ++j)
      dst[j] = plane_sy(j) < 0 ? load(j, rb, fb) : load(j, ra, fa);
    halo = bload<T>(rin, hoff + (uint32_t)(k * nx) * es, 0);
  };

  T ring[kPrefetch][kHalfPlanes];
  T hring[kPrefetch];
  auto row = [&](int k, const T *cur, const T hcur, T *refill, T &hrefill) {
    if (k + kPrefetch - 1 < yend) issue(k + kPrefetch - 1, refill, hrefill);
    const int rk = k * nx;
    SpC *sp = launder(as_const(I.sp));
    SpC &me = sp[s];
    T h1[kHalfXPlanes], h2[kHalfXPlanes];
#pragma unroll
    for (int j = 0; j < kHalfXPlanes; ++j) {
      if constexpr (kHaloGather<T>) {
        h1[j] = bperm(hidx1 + 12 * j, hcur);
        h2[j] = bperm(4 + 12 * j, hcur);
      } else {
        h1[j] = lane == 0 ? readlane(hcur, 3 * j) : readlane(hcur, 3 * j + 2);
        h2[j] = readlane(hcur, 3 * j + 1);
      }
    }
    T cgx[2], cgy[2];
#pragma unroll
    for (int lg = 0; lg < 2; ++lg) {
      cgx[lg] = Tab<T>::cgx(me, 2 * h + lg);
      cgy[lg] = Tab<T>::cgy(me, 2 * h + lg);
    }
    // Own orbit parts and partial moments to LDS; one barrier.
    T (*ob)[kWave] = orb[k & 1][s];
    double(*pb)[S][2][kWave] = pm[k & 1];
    {
      T lA[2], lB[2], lX[2], lY[2];
#pragma unroll
      for (int lg = 0; lg < 2; ++lg) {
        const T c0 = c[4 * lg], c1 = c[4 * lg + 1], c2 = c[4 * lg + 2], c3 = c[4 * lg + 3];
        const T s02 = c0 + c2, s13 = c1 + c3;
        lA[lg] = s02 + s13;
        lB[lg] = s02 - s13;
        if (lg == 0) {
          lX[lg] = c0 - c2; lY[lg] = c1 - c3;
        } else {
          lX[lg] = (c0 + c3) - (c1 + c2); lY[lg] = (c0 + c1) - (c2 + c3);
        }
      }
      double pn = 0.0, pjx = 0.0, pjy = 0.0, pE = 0.0;
#pragma unroll
      for (int lg = 0; lg < 2; ++lg) {
        const int g = 2 * h + lg;
        const double a = (double)lA[lg];
        pn += a;
        pjx = fma(me.vg[g], (double)lX[lg], pjx);
        pjy = fma(me.vg[g], (double)lY[lg], pjy);
        pE = fma(me.qg[g], a, pE);
        ob[0 * 4 + g][lane] = lA[lg];
        ob[1 * 4 + g][lane] = lB[lg];
        ob[2 * 4 + g][lane] = lX[lg];
        ob[3 * 4 + g][lane] = lY[lg];
      }
      pb[0][s][h][lane] = pn;
      pb[1][s][h][lane] = pjx;
      pb[2][s][h][lane] = pjy;
      pb[3][s][h][lane] = pE;
    }
    __syncthreads();
    T oA[4], oB[4], oX[4], oY[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      oA[g] = ob[0 * 4 + g][lane];
      oB[g] = ob[1 * 4 + g][lane];
      oX[g] = ob[2 * 4 + g][lane];
      oY[g] = ob[3 * 4 + g][lane];
    }
    auto mom = [&](int q, int sp_) { return pb[q][sp_][0][lane] + pb[q][sp_][1][lane]; };
    const double n0 = mom(0, s), jx0 = mom(1, s), jy0 = mom(2, s), E0 = mom(3, s);
    T fnv[kHalfPlanes];
    if constexpr (RKC) {
#pragma unroll
      for (int j = 0; j < kHalfPlanes; ++j)
        fnv[j] = bload<T>(rfn, (uint32_t)(rk + lcol) * es, pob + j * plb);
    }
    CellState cs;
    cell_chain<T, S>(I, sp, mom, cs);
    double dn_own = cs.dn[0];
#pragma unroll
    for (int q = 1; q < S; ++q)
      if (q == s) dn_own = cs.dn[q];
    T d[16], df[kHalfPlanes];
    collision_rhs<T>(I, me, oA, oB, oX, oY, n0, jx0, jy0, E0, n0 + dn_own, cs.ux, cs.uy,
                     cs.Tst, d);
    block_feq_pair<T>(me, d, 2 * h, df);
    const T om = Tab<T>::omega(me);
    T res[kHalfPlanes];
#pragma unroll
    for (int j = 0; j < kHalfPlanes; ++j) {
      const int lg = j >> 2, sx = plane_sx(j), sy = plane_sy(j);
      const T f = c[j];
      T a = f;
      if (sx != 0) {
        const int jx = xplane_index(j);
        const T dl = f - h1[jx];
        const T e = sx > 0 ? h1[jx] - h2[jx] : h2[jx] - h1[jx];
        const T dp = shl1e(f, h1[jx]) - f;
        T Dx;
        if (sx > 0) {
          const T sle = slope_pos<LIM>(e, dl);
          const T d0 = shr1e(dp, dl);
          const T sl = slope_pos<LIM>(d0, dp);
          Dx = fma(T(0.5), sl - shr1e(sl, sle), d0);
        } else {
          const T sle = slope_neg<LIM>(dl, dp);
          const T dhi = shl1e(dp, e);
          const T sl = slope_neg<LIM>(dp, dhi);
          Dx = fma(T(-0.5), sl - shr1e(sl, sle), dp);
        }
        a = (sx > 0) ? fma(-cgx[lg], Dx, a) : fma(cgx[lg], Dx, a);
      }
      const T fnew = cur[j];
      if (sy > 0) {
        const T dn = fnew - f;
        const T sk = slope_pos<LIM>(y1[j], dn);
        const T Dy = y1[j] + T(0.5) * (sk - y2[j]);
        a = fma(-cgy[lg], Dy, a);
        c[j] = fnew;
        y1[j] = dn;
        y2[j] = sk;
      } else if (sy < 0) {
        const T n1 = y1[j];
        const T dlo = n1 - f, dhi = fnew - n1;
        const T tk1 = slope_neg<LIM>(dlo, dhi);
        const T Dy = dlo - T(0.5) * (tk1 - y2[j]);
        a = fma(cgy[lg], Dy, a);
        c[j] = n1;
        y1[j] = fnew;
        y2[j] = tk1;
      } else {
        c[j] = fnew;
      }
      res[j] = fma(om, df[j], a);
      if constexpr (RKC) res[j] = fma(alpha, fnv[j] - res[j], res[j]);
    }
    if (writer) {
#pragma unroll
      for (int j = 0; j < kHalfPlanes; ++j)
        bstore(rout, res[j], (uint32_t)(rk + col) * es, pob + j * plb);
    }
  };

#pragma unroll
  for (int d = 0; d < kPrefetch - 1; ++d)
    if (y0 + d < yend) issue(y0 + d, ring[d], hring[d]);
  for (int k = y0; k < yend; k += kPrefetch) {
#pragma unroll
    for (int d = 0; d < kPrefetch; ++d) {
      if (k + d < yend)
        row(k + d, ring[d], hring[d], ring[(d + kPrefetch - 1) % kPrefetch],
            hring[(d + kPrefetch - 1) % kPrefetch]);
    }
  }
}

// Minimum resident wavefronts per SIMD requested from the register allocator.
#ifndef DBM_MIN_WAVES_F32
#define DBM_MIN_WAVES_F32 2
#endif
#ifndef DBM_MIN_WAVES_F64
#define DBM_MIN_WAVES_F64 1
#endif
template <typename T> struct Occ;
template <> struct Occ<float> { static constexpr int kMinWaves = DBM_MIN_WAVES_F32; };
template <> struct Occ<double> { static constexpr int kMinWaves = DBM_MIN_WAVES_F64; };
template <> struct Occ<f32x> { static constexpr int kMinWaves = DBM_MIN_WAVES_F64; };

// The chain wavefront's part of a tile: after the species wavefronts have
// published row y0's moments (first barrier), the chain of row k is formed
// before row k's barrier, from moments published before row k-1's barrier
// (NM slots of moments, row k in slot k % NM).  One barrier per row plus the
// first, as in fused_tile with CW.
template <typename T, int S, int NM = 2>
__device__ __forceinline__ void chain_tile(const InstDev &I, int y0, int rows,
                                           double (*mom)[4 * S][kWave],
                                           double (*chn)[kChainRows<S, true>][kWave]) {
  const int lane = threadIdx.x & (kWave - 1);
  __syncthreads();   // row y0's moments published
  const int nrun = rows_run(kSteadyRows<T>, rows);
  for (int k = y0; k < y0 + nrun; ++k) {
    SpC *sp = launder(as_const(I.sp));
    double(*mb)[kWave] = mom[k % NM];
    CellState cs;
    cell_chain<T, S>(I, sp, [&](int q, int sp_) { return mb[q * S + sp_][lane]; }, cs);
    double(*cb)[kWave] = chn[k & 1];
    cb[0][lane] = cs.ux;
    cb[1][lane] = cs.uy;
    cb[2][lane] = cs.Tst;
#pragma unroll
    for (int q = 0; q < S; ++q) cb[3 + q][lane] = cs.dn[q];
    __syncthreads();   // row k's barrier
  }
}

// One workgroup = S wavefronts, wavefront w advancing species w of a tile
// (plus the chain wavefront, index S, with CW); tiles are taken
// persistently from the table in XCD-grouped order.
template <typename ST, int S, int LIM, bool RKC, bool PIPE, bool SR, bool CW>
__global__ __launch_bounds__(kWave * (S + (CW ? 1 : 0)), Occ<ST>::kMinWaves) void k_fused_stage(
    const InstDev *__restrict__ insts, const Tile *__restrict__ tiles, int ntiles, int in_idx,
    int fn_idx, int out_idx, typename Stor<ST>::C alpha, int remap, uint32_t *ctr) {
  __shared__ double mom[2][4 * S][kWave];
  __shared__ double chn[CW ? 2 : 1][kChainRows<S, CW>][kWave];
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  constexpr bool kSR = SR && std::is_same<ST, float>::value;
  uint32_t step = 0;
  if constexpr (kSR) step = __hip_atomic_load(&ctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile t = tiles[remap ? xcd_remap(v, ntiles) : v];
    if (CW && s == S) {
      if constexpr (CW) chain_tile<typename Stor<ST>::C, S>(insts[t.inst], t.y0, t.rows, mom, chn);
    } else {
      fused_tile<ST, S, LIM, RKC, PIPE, SR, CW>(insts[t.inst], s, t.x0, t.y0, t.rows, in_idx,
                                                fn_idx, out_idx, alpha, step, mom, chn);
    }
    __syncthreads();
  }
  if constexpr (kSR) advance_step_counter(ctr, step, gridDim.x);
}

#ifndef DBM_MIN_WAVES_SPLIT_F32
#define DBM_MIN_WAVES_SPLIT_F32 3
#endif
#ifndef DBM_MIN_WAVES_SPLIT_F64
#define DBM_MIN_WAVES_SPLIT_F64 1
#endif
template <typename T> struct OccSplit;
template <> struct OccSplit<float> { static constexpr int kMinWaves = DBM_MIN_WAVES_SPLIT_F32; };
template <> struct OccSplit<double> { static constexpr int kMinWaves = DBM_MIN_WAVES_SPLIT_F64; };

// Split form: one workgroup = 2S wavefronts, wavefront 2s+h advancing half h
// of species s of a tile.
template <typename T, int S, int LIM, bool RKC>
__global__ __launch_bounds__(kWave * 2 * S, OccSplit<T>::kMinWaves) void k_fused_split(
    const InstDev *__restrict__ insts, const Tile *__restrict__ tiles, int ntiles, int in_idx,
    int fn_idx, int out_idx, T alpha, T beta, int remap) {
  __shared__ T orb[2][S][16][kWave];
  __shared__ double pm[2][4][S][2][kWave];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int s = w >> 1, h = w & 1;
  (void)beta;
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile t = tiles[remap ? xcd_remap(v, ntiles) : v];
    fused_tile_split<T, S, LIM, RKC>(insts[t.inst], s, h, t.x0, t.y0, t.rows, in_idx, fn_idx,
                                     out_idx, alpha, orb, pm);
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// OM storage of FP32-bulk f (see SpeciesDev): per cell and species the
// A-block moments of f - fref and the orbit components B, X, Y of f.
//
// Storing f_i itself in FP32 rounds each value to 2^-24 of its size, so the
// momentum sum_i f_i v_i and the mass and energy carry rounding noise of
// order 2^-24 |f| c per step whatever the flow speed is.  Stored this way,
// the mass and energy are kept as differences from a fixed reference state
// and the momentum as the signed orbit sums X, Y, each rounded relative to its
// own size: near rest and near the reference the noise shrinks with the
// deviation.  The representation is a fixed invertible linear map of f, so
// each update is formed as an increment in the same basis (from the
// convection of the reconstructed f - fref and the moment-space collision)
// and added to the stored values with one rounding.
// ---------------------------------------------------------------------------

// Slot pattern of a specular reflection in y (v_y -> -v_y): the diagonal
// groups' B and every Y change sign, the rest is invariant.
__host__ __device__ constexpr bool om_odd_in_y(int k) {
  return k == 5 || k == 7 || k >= 12;
}
__device__ __forceinline__ void om_flip(float *s, bool flip) {
  if (flip) {
#pragma unroll
    for (int k = 0; k < kNV; ++k)
      if (om_odd_in_y(k)) s[k] = -s[k];
  }
}

// f - fref (plane order of Eq.15) from the stored values, FP32 arithmetic:
// a_g = A_g / 4 from the A-block moments, then each group from a, B, X, Y.
__device__ __forceinline__ void om_recon(SpC &sp, const float *s, float *f) {
  const float DBM_CONST *KA = sp.KA_f;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float al = KA[g * 4] * s[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) al = fma(KA[g * 4 + j], s[j], al);
    const float B = s[4 + g], X = s[8 + g], Y = s[12 + g];
    const float p = fma(0.25f, B, al), m = fma(-0.25f, B, al);
    float *o = f + 4 * g;
    if ((g & 1) == 0) {
      o[0] = fma(0.5f, X, p); o[1] = fma(0.5f, Y, m);
      o[2] = fma(-0.5f, X, p); o[3] = fma(-0.5f, Y, m);
    } else {
      const float sm = X + Y, df = X - Y;
      o[0] = fma(0.25f, sm, p); o[1] = fma(-0.25f, df, m);
      o[2] = fma(-0.25f, sm, p); o[3] = fma(0.25f, df, m);
    }
  }
}

// Increment of the stored values for an increment dc of f (plane order):
// orbit components of dc, and the A-block moments of its orbit sums.
__device__ __forceinline__ void om_project(SpC &sp, const float *dc, float *ds) {
  float A[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float c0 = dc[4 * g], c1 = dc[4 * g + 1], c2 = dc[4 * g + 2], c3 = dc[4 * g + 3];
    const float s02 = c0 + c2, s13 = c1 + c3;
    A[g] = s02 + s13;
    ds[4 + g] = s02 - s13;
    if ((g & 1) == 0) {
      ds[8 + g] = c0 - c2; ds[12 + g] = c1 - c3;
    } else {
      ds[8 + g] = (c0 + c3) - (c1 + c2); ds[12 + g] = (c0 + c1) - (c2 + c3);
    }
  }
  const float DBM_CONST *MA = sp.MA_f;
  ds[0] = (A[0] + A[1]) + (A[2] + A[3]);
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    float m = MA[j * 4] * A[0];
#pragma unroll
    for (int g = 1; g < 4; ++g) m = fma(MA[j * 4 + g], A[g], m);
    ds[j] = m;
  }
}

// Adds the collision increment omega M^{-1} d, expressed in the stored basis,
// to ds: omega d for the A-block moments, omega (iB, iE) d for B, X, Y.
__device__ __forceinline__ void om_add_collision(SpC &sp, const float *d, float *ds) {
  const float om = sp.omega_f;
#pragma unroll
  for (int j = 0; j < 4; ++j) ds[j] = fma(om, d[j], ds[j]);
  const float DBM_CONST *B1 = sp.wB1_f;
  const float DBM_CONST *B2 = sp.wB2_f;
  ds[4] = fma(B1[1], d[5], fma(B1[0], d[4], ds[4]));
  ds[6] = fma(B1[3], d[5], fma(B1[2], d[4], ds[6]));
  ds[5] = fma(B2[1], d[7], fma(B2[0], d[6], ds[5]));
  ds[7] = fma(B2[3], d[7], fma(B2[2], d[6], ds[7]));
  const float DBM_CONST *E = sp.wE_f;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float x = ds[8 + g], y = ds[12 + g];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x = fma(E[g * 4 + j], d[8 + j], x);
      y = fma(E[g * 4 + j], d[12 + j], y);
    }
    ds[8 + g] = x;
    ds[12 + g] = y;
  }
}

// FP64 species moments from the stored values: n and E are the first two
// A-block moments plus the reference's, j = sum_g v_g (X_g, Y_g).
template <typename P>
__device__ __forceinline__ void om_moments(SpC &sp, P sref, const float *s, double &n,
                                           double &jx, double &jy, double &E) {
  n = (double)s[0] + sref[0];
  E = (double)s[1] + sref[1];
  jx = jy = 0.0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    jx = fma(sp.vg[g], (double)s[8 + g], jx);
    jy = fma(sp.vg[g], (double)s[12 + g], jy);
  }
}

// g - M f of one species in the order of eq_rhs (collision_rhs on OM
// storage): the conserved rows 0, 1, 8, 12 and the A-block rows 2, 3 are
// differenced in FP64 against the stored moments plus the reference's; the
// B, X and Y rows in FP32, where both terms are small near rest.
template <typename P>
__device__ __forceinline__ void collision_rhs_om(const InstDev &I, SpC &sp, P sref,
                                                 const float *s,
                                                 double n, double jx, double jy, double E,
                                                 double ns, double ux, double uy, double Tst,
                                                 float *d) {
  const double K = sp.K, th = Tst * sp.inv_m, u2 = ux * ux + uy * uy;
  float r[16];
  eq_rhs<float>((float)ns, (float)ux, (float)uy, (float)th, (float)K, r);
  const double e2 = (K + 2.0) * th + u2, e4 = (K + 4.0) * th + u2;
  double d0 = ns - n, d1 = ns * fma(K, th, u2) - E, d8 = ns * ux - jx, d12 = ns * uy - jy;
  double d2 = (ns * (2.0 * th + u2) - sref[2]) - (double)s[2];
  double d3 = (ns * fma(2.0 * th, e2, u2 * e4) - sref[3]) - (double)s[3];
  const bool force = I.force && n > 1e-300;
  double fd[16];
  if (force) {
    const double inv_n = recip<float>(n);
    const double us = jx * inv_n, vs = jy * inv_n;
    const double Ts = sp.m * (E * inv_n - us * us - vs * vs) * sp.inv_K;
    double Td = Ts;
    if (I.fmode == DBM_FORCE_T_EXACT)
      Td = Ts - sp.m * sp.tau * sp.tau * (I.ax * I.ax + I.ay * I.ay) * sp.inv_K;
    double r1[16], r2[16];
    eq_rhs<double>(n, us + sp.tau * I.ax, vs + sp.tau * I.ay, Td * sp.inv_m, K, r1);
    eq_rhs<double>(n, us, vs, Ts * sp.inv_m, K, r2);
#pragma unroll
    for (int k = 0; k < 16; ++k) fd[k] = r1[k] - r2[k];
    d0 += fd[0];
    d1 += fd[1];
    d2 += fd[2];
    d3 += fd[3];
    d8 += fd[8];
    d12 += fd[12];
  }
  const float DBM_CONST *MB1 = launder_after(sp.MB1_f, r[4]);
  const float DBM_CONST *MB2 = launder_after(sp.MB2_f, r[6]);
  const float DBM_CONST *ME = launder_after(sp.ME_f, r[9]);
  d[0] = (float)d0;
  d[1] = (float)d1;
  d[2] = (float)d2;
  d[3] = (float)d3;
  d[8] = (float)d8;
  d[12] = (float)d12;
  d[4] = r[4] - fma(MB1[1], s[6], MB1[0] * s[4]);
  d[5] = r[5] - fma(MB1[3], s[6], MB1[2] * s[4]);
  d[6] = r[6] - fma(MB2[1], s[7], MB2[0] * s[5]);
  d[7] = r[7] - fma(MB2[3], s[7], MB2[2] * s[5]);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    float mx = ME[row * 4] * s[8], my = ME[row * 4] * s[12];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      mx = fma(ME[row * 4 + j], s[8 + j], mx);
      my = fma(ME[row * 4 + j], s[12 + j], my);
    }
    d[8 + row] = r[8 + row] - mx;
    d[12 + row] = r[12 + row] - my;
  }
  if (force) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k != 0 && k != 1 && k != 2 && k != 3 && k != 8 && k != 12) d[k] += (float)fd[k];
  }
}

// FP64 conversions between f and OM storage (initialisation, transfers,
// diagnostics and changes of representation).
__device__ __forceinline__ void om_pack(const SpeciesDev &sp, const double *fref, const double *f,
                                        double *s) {
  double A[4];
  for (int g = 0; g < 4; ++g) {
    const double c0 = f[4 * g] - fref[4 * g], c1 = f[4 * g + 1] - fref[4 * g + 1];
    const double c2 = f[4 * g + 2] - fref[4 * g + 2], c3 = f[4 * g + 3] - fref[4 * g + 3];
    A[g] = (c0 + c2) + (c1 + c3);
    s[4 + g] = (c0 + c2) - (c1 + c3);
    if ((g & 1) == 0) {
      s[8 + g] = c0 - c2;
      s[12 + g] = c1 - c3;
    } else {
      s[8 + g] = (c0 + c3) - (c1 + c2);
      s[12 + g] = (c0 + c1) - (c2 + c3);
    }
  }
  for (int j = 0; j < 4; ++j) {
    double m = 0.0;
    for (int g = 0; g < 4; ++g) m = fma(sp.MA[j * 4 + g], A[g], m);
    s[j] = m;
  }
}
// The stored FP32 values, and with `lo` the A-block residuals.
__device__ __forceinline__ void om_pack(const SpeciesDev &sp, const double *fref, const double *f,
                                        float *s, uint16_t *lo = nullptr) {
  double d[kNV];
  om_pack(sp, fref, f, d);
  for (int i = 0; i < kNV; ++i) s[i] = (float)d[i];
  if (lo)
    for (int j = 0; j < 4; ++j) split_f32x(d[j], s[j], lo[j]);
}
template <typename V>
__device__ __forceinline__ void om_unpack(const SpeciesDev &sp, const double *fref, const V *s,
                                          double *f) {
  for (int g = 0; g < 4; ++g) {
    double A = 0.0;
    for (int j = 0; j < 4; ++j) A = fma(sp.iA[g * 4 + j], (double)s[j], A);
    const double B = s[4 + g], X = s[8 + g], Y = s[12 + g];
    const double p = 0.25 * (A + B), m = 0.25 * (A - B);
    double *o = f + 4 * g;
    if ((g & 1) == 0) {
      o[0] = p + 0.5 * X; o[1] = m + 0.5 * Y; o[2] = p - 0.5 * X; o[3] = m - 0.5 * Y;
    } else {
      const double sm = 0.25 * (X + Y), df = 0.25 * (X - Y);
      o[0] = p + sm; o[1] = m - df; o[2] = p - sm; o[3] = m + df;
    }
    for (int k = 0; k < 4; ++k) o[k] += fref[4 * g + k];
  }
}

// The OM reference of species s at grid row y: fref (16 FP64 values) and its
// A-block moments sref (4 more).
__device__ __forceinline__ const double *om_rowref(const InstDev &I, int s, int y) {
  return I.rref + ((size_t)s * I.ny + y) * kRowRef;
}
// The same for the one-pass kernel, where s and y are wave-uniform: read
// through the constant address space (scalar loads), re-read at each use.
__device__ __forceinline__ const double DBM_CONST *om_rowref_c(const InstDev &I, int s, int y) {
  return launder((const double DBM_CONST *)om_rowref(I, s, y));
}

// DPP broadcasts used by the halo transform: row_newbcast:n gives every lane
// of a 16-lane row the value of lane n of that row; quad_perm [q,q,q,q] the
// value of lane q of its quad.
template <int N> __device__ __forceinline__ float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + N, 0xf, 0xf, false));
}
template <int Q> __device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(v), Q | (Q << 2) | (Q << 4) | (Q << 6), 0xf, 0xf, false));
}

// Rows of loads in flight per wavefront (OM form).
#ifndef DBM_OM_RING
#define DBM_OM_RING 2
#endif
constexpr int kRingOM = DBM_OM_RING;
static_assert(kRingOM >= 2, "the prefetch ring needs two or more slots");

// The per-wavefront hold of stored rows: row r's 16 stored values sit in
// slot r % 3 from the time they are loaded (two rows ahead, for the
// stencil's look-ahead) until row r's own update, as four float4 per lane.
typedef float float4_t __attribute__((ext_vector_type(4)));
constexpr int kHoldRows = 3;

// s_waitcnt immediate (gfx9 encoding) that waits for every vector memory
// operation of the wavefront (vmcnt 0) and for nothing else.
constexpr int kWaitVmem0 = 0x0F70;

// One wavefront's share of a tile on OM storage (FP32-bulk): species `s`,
// 64 lanes = columns x0 .. x0+63, rows y0 .. y0+rows-1, marching in +y.
//  * Stored row r arrives two rows ahead (the look-ahead of planes with
//    v_y < 0), is reconstructed to f - fref once (the planes with v_y >= 0
//    keep it for one more row) and parked in the hold until row r is updated.
//  * The x-halo (columns x0-2, x0-1, x0+64, x0+65) arrives as one load of
//    all 16 stored values of those four cells (lane 16 w + 4 g + q: column w,
//    slot 4 q + g) and is turned into f - fref by two rounds of DPP
//    broadcasts: the A-block moments into a_g within each 16-lane row, then
//    a, B, X, Y into the group's four planes within each quad (lane 16 w + i:
//    plane i at column w).  The edge lanes then gather it as in fused_tile.
//  * The update of row k is formed in the stored basis: the stencil
//    increment projected onto it plus the moment-space collision, added to
//    row k's stored values with one rounding.
//  * With A-block residuals (AR) the four A-block values are summed in FP64
//    with their residuals (loaded at the row's start) and stored as FP32
//    plus a new residual: the stencils and the collision see the FP32
//    values, the sum keeps what their rounding would drop each step.
template <int S, int LIM, bool RKC, bool SR, bool CW, bool RR, bool AR>
__device__ __forceinline__ void fused_tile_om(const InstDev &I, const int s, int x0, int y0,
                                              int rows, int in_idx, int fn_idx, int out_idx,
                                              float alpha, uint32_t step, int drain,
                                              double (*mom)[4 * S][kWave],
                                              double (*chn)[kChainRows<S, CW>][kWave],
                                              float4_t (*hold)[4][kWave], float (*hhold)[kWave]) {
  // mom: two slots (row parity) without the chain wavefront, three with it
  typedef float T;
  constexpr int kPf = kRingOM;
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = I.nx, ny = I.ny, bcy = I.bcy;
  const FBuf<float> bin(I, in_idx, s), bfn(I, fn_idx, s), bout(I, out_idx, s);
  const int col = x0 + lane;
  const int lcol = map_x(col, nx, I.bcx);
  const bool writer = col < nx;
  const int yend = y0 + rows;
  static_assert(!(AR && SR), "A-block residuals are summed with round to nearest");

  auto hold_put = [&](int r, const T *v) {
    float4_t(*h)[kWave] = hold[r % kHoldRows];
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q][lane] = float4_t{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
  };
  auto hold_get = [&](int r, T *v) {
    float4_t(*h)[kWave] = hold[r % kHoldRows];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4_t w = h[q][lane];
      v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
    }
  };
  // Stored row r at this lane's column (reflected rows: see om_flip).
  auto load_row = [&](int r, T *dst, bool &flip) {
    const int rr = map_y(r, ny, bcy, flip) * nx;
#pragma unroll
    for (int i = 0; i < kNV; ++i) dst[i] = bin.value((uint32_t)(rr + lcol), i);
  };
  // Chain wavefront: row r's FP64 moments from its stored values, published
  // as soon as they arrive (row r in slot r % 3 of the moment exchange).
  auto publish = [&](SpC &me, int r, const T *sv) {
    double n, jx, jy, E;
    if constexpr (RR) om_moments(me, om_rowref_c(I, s, r) + kNV, sv, n, jx, jy, E);
    else om_moments(me, (const double DBM_CONST *)me.sref, sv, n, jx, jy, E);
    double(*mb)[kWave] = mom[r % 3];
    mb[0 * S + s][lane] = n;
    mb[1 * S + s][lane] = jx;
    mb[2 * S + s][lane] = jy;
    mb[3 * S + s][lane] = E;
  };

  // Halo lanes: lane 16 w + 4 g + q reads slot 4 q + g of column w.
  const int hw = lane >> 4, hg = (lane >> 2) & 3, hq = lane & 3;
  const uint32_t hplane = (uint32_t)(4 * hq + hg);
  uint32_t hcol;
  {
    const int c = hw == 0 ? x0 - 2 : (hw == 1 ? x0 - 1 : (hw == 2 ? x0 + kWave : x0 + kWave + 1));
    hcol = (uint32_t)map_x(c, nx, I.bcx);
  }
  // Transform coefficients.  Round 1 (A-block moments -> a_g, in the lanes
  // with q = 0; the others keep their value): a = own * hown + sum_j hcA[j] *
  // (slot j of the row).  Round 2 (plane 4 g + c from a_g, B_g, X_g, Y_g):
  // coefficients 1, hcB, hcX, hcY.
  T hown, hcA[4], hcB, hcX, hcY;
  {
    SpC &me = launder(as_const(I.sp))[s];
    hown = hq == 0 ? 0.f : 1.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T k0 = me.KA_f[j], k1 = me.KA_f[4 + j], k2 = me.KA_f[8 + j], k3 = me.KA_f[12 + j];
      const T kg = hg == 0 ? k0 : (hg == 1 ? k1 : (hg == 2 ? k2 : k3));
      hcA[j] = hq == 0 ? kg : 0.f;
    }
    const int c = hq;
    hcB = (c & 1) ? -0.25f : 0.25f;
    if ((hg & 1) == 0) {          // axis group: planes +x, +y, -x, -y
      hcX = c == 0 ? 0.5f : (c == 2 ? -0.5f : 0.f);
      hcY = c == 1 ? 0.5f : (c == 3 ? -0.5f : 0.f);
    } else {                      // diagonal group: (1,1), (-1,1), (-1,-1), (1,-1)
      hcX = (c == 0 || c == 3) ? 0.25f : -0.25f;
      hcY = (c == 0 || c == 1) ? 0.25f : -0.25f;
    }
  }
  const int hidx1 = lane == kWave - 1 ? 32 * 4 : 16 * 4;
  // The raw halo of row r is loaded together with stored row r (two rows
  // ahead, when the tile to the left or right loads the same cache lines as
  // its own row r) and parked in slot r % 3 of hhold until row r's update.
  auto halo_load = [&](int r) { return bin.lane_value(hplane, hcol + (uint32_t)(r * nx)); };

  // fref(row r+1) - fref(row r), one value per velocity group (the planes of
  // a group are equal at rest): the stencil's differences between rows are
  // formed from the stored deviations and this.  Rows r and r+1 are read
  // together (scalar loads) at the start of row r's update.
  const float *dref = I.dref + (size_t)s * (ny + 4) * 4;
  auto dref_rows = [&](int r, float *d0, float *d1) {
    const float DBM_CONST *p = launder((const float DBM_CONST *)(dref + (size_t)(r + 2) * 4));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      d0[g] = p[g];
      d1[g] = p[4 + g];
    }
  };

  // Rows y0-2 .. y0+1: the stencil state of row y0 and the first two rows
  // of the hold.
  T c[kNV], y1[kNV], y2[kNV], nxv[kNV];
  {
    SpC &me = launder(as_const(I.sp))[s];
    T sa[kNV], sb[kNV], s0[kNV], s1[kNV];
    bool fa, fb, f0, f1;
    load_row(y0 - 2, sa, fa);
    load_row(y0 - 1, sb, fb);
    load_row(y0, s0, f0);
    load_row(y0 + 1, s1, f1);
    om_flip(sa, fa);
    om_flip(sb, fb);
    om_flip(s1, f1);
    hold_put(y0, s0);
    hhold[y0 % kHoldRows][lane] = halo_load(y0);
    if (y0 + 1 < yend) {
      hold_put(y0 + 1, s1);
      hhold[(y0 + 1) % kHoldRows][lane] = halo_load(y0 + 1);
    }
    T ra[kNV], rb[kNV], r1[kNV];
    om_recon(me, sa, ra);
    om_recon(me, sb, rb);
    om_recon(me, s0, c);
    om_recon(me, s1, r1);
    float da[4] = {0.f, 0.f, 0.f, 0.f}, db[4] = {0.f, 0.f, 0.f, 0.f}, d0[4] = {0.f, 0.f, 0.f, 0.f},
          dn[4];
    if constexpr (RR) {
      dref_rows(y0 - 2, da, db);
      dref_rows(y0, d0, dn);
    }
#pragma unroll
    for (int i = 0; i < kNV; ++i) {
      const int sy = plane_sy(i);
      if (sy > 0) {
        y1[i] = RR ? (c[i] - rb[i]) + db[i >> 2] : c[i] - rb[i];
        y2[i] = slope_pos<LIM>(RR ? (rb[i] - ra[i]) + da[i >> 2] : rb[i] - ra[i], y1[i]);
        nxv[i] = r1[i];
      } else if (sy < 0) {
        y1[i] = r1[i];
        y2[i] = slope_neg<LIM>(RR ? (c[i] - rb[i]) + db[i >> 2] : c[i] - rb[i],
                               RR ? (r1[i] - c[i]) + d0[i >> 2] : r1[i] - c[i]);
        nxv[i] = T(0);
      } else {
        y1[i] = y2[i] = T(0);
        nxv[i] = r1[i];
      }
    }
    if constexpr (CW) {   // rows y0 and y0+1 for the chain wavefront's first chains
      publish(me, y0, s0);
      if (y0 + 1 < yend) publish(me, y0 + 1, s1);
      __syncthreads();
    }
  }

  // Ring slot of time t: stored row t+2 (with its reflection flag) and its
  // raw halo.  Every row issues its refill without a branch around it (past
  // the tile's end the slot takes a row again, unused, and a halo row that
  // is not updated is replaced by the tile's last, loaded and not parked):
  // the compiler's count of loads in flight then stays exact, and the wait
  // for the row that arrived leaves the loads issued after it in flight.
  // (RK3 stages, which also hold f^n, keep the branches at the tile's end:
  // without them the compiler's schedule does not fit their registers.)
  auto issue = [&](int t, T *dst, T &halo, bool &flip) {
    if constexpr (RKC) {
      load_row(t + 2, dst, flip);
      halo = t + 2 < yend ? halo_load(t + 2) : T(0);
    } else {
      t = t < yend ? t : yend - 1;
      load_row(t + 2, dst, flip);
      halo = halo_load(t + 2 < yend ? t + 2 : yend - 1);
    }
  };
  T ring[kPf][kNV];
  T hring[kPf];
  bool rflip[kPf];
#pragma unroll
  for (int d = 0; d < kPf - 1; ++d) issue(y0 + d, ring[d], hring[d], rflip[d]);

  auto row = [&](int k, const T *cur, const T hcur, const bool cflip, T *refill, T &hrefill,
                 bool &rfl) {
    if constexpr (RKC) {
      if (k + kPf - 1 < yend) issue(k + kPf - 1, refill, hrefill, rfl);
    } else {
      issue(k + kPf - 1, refill, hrefill, rfl);
      // drain (a form the autotuner times against the other): every other
      // row waits for its refill at once, which halves the loads in flight.
      if (drain && ((k - y0) & 1) == 0) __builtin_amdgcn_s_waitcnt(kWaitVmem0);
    }
    const int rk = k * nx;
    // With references per row: this row's reference differences (rows k,
    // k+1) and moments, scalar loads issued at the row's start and used by
    // its stencils and collision.  With one reference for the grid the
    // differences vanish and the moments are read where they are used.
    // A-block residuals of row k (and of f^n for the combine).
    uint16_t rlo[4], rfn[4];
    if constexpr (AR) {
      const AResBuf ain(I, in_idx, s);
#pragma unroll
      for (int j = 0; j < 4; ++j) rlo[j] = ain.value((uint32_t)(rk + lcol), j);
    }
    float dk[4], dk1[4];
    double sref_row[4];
    if constexpr (RR) {
      dref_rows(k, dk, dk1);
      const double DBM_CONST *srp = om_rowref_c(I, s, k) + kNV;
#pragma unroll
      for (int j = 0; j < 4; ++j) sref_row[j] = srp[j];
    }
    SpC *sp = launder(as_const(I.sp));
    SpC &me = sp[s];
    auto sref_k = [&]() {
      if constexpr (RR) return (const double *)sref_row;
      else return (const double DBM_CONST *)me.sref;
    };
    // Stored row k+2: hold it for its own update, reconstruct it for the
    // stencil (planes with v_y < 0 now, the others next row).
    T fnew[kNV];
    {
      T sn[kNV];
#pragma unroll
      for (int i = 0; i < kNV; ++i) sn[i] = cur[i];
      om_flip(sn, cflip);
      if (k + 2 < yend) {
        hold_put(k + 2, sn);
        hhold[(k + 2) % kHoldRows][lane] = hcur;
        if constexpr (CW) publish(me, k + 2, sn);
      }
      om_recon(me, sn, fnew);
    }
    T nv[kNV];
#pragma unroll
    for (int i = 0; i < kNV; ++i) {
      if (plane_sy(i) < 0) {
        nv[i] = fnew[i];
      } else {
        nv[i] = nxv[i];
        nxv[i] = fnew[i];
      }
    }
    // Collision of row k from its stored values (into sk, d).  With the
    // chain wavefront it comes before the stencils (the chain is ready at the
    // row's barrier, and the stencils' registers are free then: no spills);
    // without it after them (measured faster for four species, where each
    // wavefront forms the chain after the barrier).
    T sk[kNV];
    T d[kNV];
    if constexpr (CW) {
      hold_get(k, sk);
      double n0, jx0, jy0, E0;
      om_moments(me, sref_k(), sk, n0, jx0, jy0, E0);
      __syncthreads();
      double(*cb)[kWave] = chn[k & 1];
      const double ux = cb[0][lane], uy = cb[1][lane], Tst = cb[2][lane], dn = cb[3 + s][lane];
      collision_rhs_om(I, me, sref_k(), sk, n0, jx0, jy0, E0, n0 + dn, ux, uy, Tst, d);
    }
    // x-halo of row k as f - fref, and its gathers to the edge lanes.
    T hf;
    {
      const T hk = hhold[k % kHoldRows][lane];
      T a = hown * hk;
      a = fma(hcA[0], row_bcast<0>(hk), a);
      a = fma(hcA[1], row_bcast<4>(hk), a);
      a = fma(hcA[2], row_bcast<8>(hk), a);
      a = fma(hcA[3], row_bcast<12>(hk), a);
      hf = quad_bcast<0>(a);
      hf = fma(hcB, quad_bcast<1>(a), hf);
      hf = fma(hcX, quad_bcast<2>(a), hf);
      hf = fma(hcY, quad_bcast<3>(a), hf);
    }
    T h1[kXPlanes], h2[kXPlanes];
#pragma unroll
    for (int j = 0; j < kXPlanes; ++j) {
      const int i = xplane(j);
      h1[j] = bperm(hidx1 + 4 * i, hf);
      h2[j] = bperm(4 * (plane_sx(i) > 0 ? i : 48 + i), hf);
    }
    T cgx[4], cgy[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      cgx[g] = me.cgx_f[g];
      cgy[g] = me.cgy_f[g];
    }
    // Stencil increments of row k (NND in x from adjacent lanes and the
    // halo, in y from the carried rows); advances the carried state.
    T dc[kNV];
#pragma unroll
    for (int i = 0; i < kNV; ++i) {
      const int g = i >> 2, sx = plane_sx(i), sy = plane_sy(i);
      const T f = c[i];
      T a = T(0);
      if (sx != 0) {
        const int j = xplane_index(i);
        const T dl = f - h1[j];
        const T e = sx > 0 ? h1[j] - h2[j] : h2[j] - h1[j];
        const T dp = shl1e(f, h1[j]) - f;
        T Dx;
        if (sx > 0) {
          const T sle = slope_pos<LIM>(e, dl);
          const T d0 = shr1e(dp, dl);
          const T sl = slope_pos<LIM>(d0, dp);
          Dx = fma(T(0.5), sl - shr1e(sl, sle), d0);
          a = -cgx[g] * Dx;
        } else {
          const T sle = slope_neg<LIM>(dl, dp);
          const T dhi = shl1e(dp, e);
          const T sl = slope_neg<LIM>(dp, dhi);
          Dx = fma(T(-0.5), sl - shr1e(sl, sle), dp);
          a = cgx[g] * Dx;
        }
      }
      const T fn = nv[i];
      if (sy > 0) {
        const T dn = RR ? (fn - f) + dk[g] : fn - f;
        const T sk = slope_pos<LIM>(y1[i], dn);
        const T Dy = y1[i] + T(0.5) * (sk - y2[i]);
        a = fma(-cgy[g], Dy, a);
        c[i] = fn;
        y1[i] = dn;
        y2[i] = sk;
      } else if (sy < 0) {
        const T n1 = y1[i];
        const T dlo = RR ? (n1 - f) + dk[g] : n1 - f;
        const T dhi = RR ? (fn - n1) + dk1[g] : fn - n1;
        const T tk1 = slope_neg<LIM>(dlo, dhi);
        const T Dy = dlo - T(0.5) * (tk1 - y2[i]);
        a = fma(cgy[g], Dy, a);
        c[i] = n1;
        y1[i] = fn;
        y2[i] = tk1;
      } else {
        c[i] = fn;
      }
      dc[i] = a;
    }
    // f^n of the Runge-Kutta combine, requested before the moment exchange
    // and the collision so that their latency hides behind them (with the
    // chain wavefront the registers for that are not there: requested with
    // the combine).
    constexpr bool kEarlyFn = RKC && !CW;
    const int rkn = k < ny ? rk : (ny - 1) * nx;
    T fnv[kNV];
    if constexpr (kEarlyFn) {
#pragma unroll
      for (int i = 0; i < kNV; ++i) fnv[i] = bfn.value((uint32_t)(rkn + lcol), i);
    }
    if constexpr (!CW) {
      hold_get(k, sk);
      double n0, jx0, jy0, E0;
      om_moments(me, sref_k(), sk, n0, jx0, jy0, E0);
      double ux, uy, Tst, dn;
      double(*mb)[kWave] = mom[k & 1];
      mb[0 * S + s][lane] = n0;
      mb[1 * S + s][lane] = jx0;
      mb[2 * S + s][lane] = jy0;
      mb[3 * S + s][lane] = E0;
      __syncthreads();
      CellState cs;
      cell_chain<T, S>(I, sp, [&](int q, int sp_) { return mb[q * S + sp_][lane]; }, cs);
      dn = cs.dn[0];
#pragma unroll
      for (int q = 1; q < S; ++q)
        if (q == s) dn = cs.dn[q];   // wave-uniform select, no indexed array
      ux = cs.ux;
      uy = cs.uy;
      Tst = cs.Tst;
      collision_rhs_om(I, me, sref_k(), sk, n0, jx0, jy0, E0, n0 + dn, ux, uy, Tst, d);
    }
    T ds[kNV];
    om_project(me, dc, ds);
    om_add_collision(me, d, ds);
    // Stage combine in the stored basis and one store per value.
    T res[kNV];
    if constexpr (SR) {
      const uint32_t key = sr_key((uint32_t)(rk + col), s, step, sk);
      uint32_t rb[4];
      rb[0] = mix32(key);
      rb[1] = mix32(key ^ 0x68E31DA4u);
      rb[2] = mix32(key ^ 0xB5297A4Du);
      rb[3] = mix32(key ^ 0x1B56C4E9u);
#pragma unroll
      for (int i = 0; i < kNV; ++i) {
        T dd = ds[i];
        if constexpr (RKC) {
          const T fn = kEarlyFn ? fnv[i] : bfn.value((uint32_t)(rkn + lcol), i);
          dd = fma(alpha, (fn - sk[i]) - dd, dd);
        }
        res[i] = sr_add(sk[i], dd, rb[i >> 2] >> (8 * (i & 3)));
      }
    } else {
      if constexpr (AR && RKC) {
        const AResBuf afn(I, fn_idx, s);
#pragma unroll
        for (int j = 0; j < 4; ++j) rfn[j] = afn.value((uint32_t)(rkn + lcol), j);
      }
#pragma unroll
      for (int i = 0; i < kNV; ++i) {
        if (AR && i < 4) {
          double v = ((double)sk[i] + (double)bf16_value(rlo[i])) + (double)ds[i];
          if constexpr (RKC) {
            const T fn = kEarlyFn ? fnv[i] : bfn.value((uint32_t)(rkn + lcol), i);
            const double fv = (double)fn + (double)bf16_value(rfn[i]);
            v = fma((double)alpha, fv - v, v);
          }
          split_f32x(v, res[i], rlo[i]);
          continue;
        }
        res[i] = sk[i] + ds[i];
        if constexpr (RKC) {
          const T fn = kEarlyFn ? fnv[i] : bfn.value((uint32_t)(rkn + lcol), i);
          res[i] = fma(alpha, fn - res[i], res[i]);
        }
      }
    }
    if (writer) {
#pragma unroll
      for (int i = 0; i < kNV; ++i) bout.store((uint32_t)(rk + col), i, res[i]);
      if constexpr (AR) {
        const AResBuf aout(I, out_idx, s);
#pragma unroll
        for (int j = 0; j < 4; ++j) aout.store((uint32_t)(rk + col), j, rlo[j]);
      }
    }
  };

  // Whole rounds of the ring in the loop (no branch around a row), the
  // rest after it.
  if constexpr (RKC) {
    for (int k = y0; k < yend; k += kPf) {
#pragma unroll
      for (int d = 0; d < kPf; ++d) {
        if (k + d < yend)
          row(k + d, ring[d], hring[d], rflip[d], ring[(d + kPf - 1) % kPf],
              hring[(d + kPf - 1) % kPf], rflip[(d + kPf - 1) % kPf]);
      }
    }
  } else {
    int k = y0;
    for (; k + kPf <= yend; k += kPf) {
#pragma unroll
      for (int d = 0; d < kPf; ++d)
        row(k + d, ring[d], hring[d], rflip[d], ring[(d + kPf - 1) % kPf],
            hring[(d + kPf - 1) % kPf], rflip[(d + kPf - 1) % kPf]);
    }
#pragma unroll
    for (int d = 0; d < kPf - 1; ++d) {
      if (k + d < yend)
        row(k + d, ring[d], hring[d], rflip[d], ring[(d + kPf - 1) % kPf],
            hring[(d + kPf - 1) % kPf], rflip[(d + kPf - 1) % kPf]);
    }
  }
}

// One workgroup = S wavefronts (plus the chain wavefront with CW), tiles
// taken persistently in XCD-grouped order, as k_fused_stage.
template <int S, int LIM, bool RKC, bool SR, bool CW, bool RR, bool AR>
__global__ __launch_bounds__(kWave * (S + (CW ? 1 : 0)), DBM_MIN_WAVES_F32) void k_fused_om(
    const InstDev *__restrict__ insts, const Tile *__restrict__ tiles, int ntiles, int in_idx,
    int fn_idx, int out_idx, float alpha, int remap, uint32_t *ctr, int drain) {
  __shared__ double mom[CW ? 3 : 2][4 * S][kWave];
  __shared__ double chn[CW ? 2 : 1][kChainRows<S, CW>][kWave];
  __shared__ float4_t hold[S][kHoldRows][4][kWave];
  __shared__ float hhold[S][kHoldRows][kWave];
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  uint32_t step = 0;
  if constexpr (SR) step = __hip_atomic_load(&ctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int v = blockIdx.x; v < ntiles; v += gridDim.x) {
    const Tile t = tiles[remap ? xcd_remap(v, ntiles) : v];
    if (CW && s == S) {
      if constexpr (CW) chain_tile<float, S, 3>(insts[t.inst], t.y0, t.rows, mom, chn);
    } else {
      fused_tile_om<S, LIM, RKC, SR, CW, RR, AR>(insts[t.inst], s, t.x0, t.y0, t.rows, in_idx, fn_idx,
                                          out_idx, alpha, step, drain, mom, chn,
                                          hold[CW && s == S ? 0 : s], hhold[CW && s == S ? 0 : s]);
    }
    __syncthreads();
  }
  if constexpr (SR) advance_step_counter(ctr, step, gridDim.x);
}

// ---------------------------------------------------------------------------
// Plain path: one thread per cell for the equilibrium (dense FP64 M^{-1}),
// one thread per (cell, plane) for convection + combine.
// ---------------------------------------------------------------------------
template <typename ST>
__device__ __forceinline__ void plain_feq_cell(const InstDev &I, const FV<ST> &f, size_t plane,
                                               size_t cell, typename Stor<ST>::C *dst) {
  typedef typename Stor<ST>::C T;
  const int S = I.S;
  const SpeciesDev *sp = I.sp;
  double n[kMaxSpecies], jx[kMaxSpecies], jy[kMaxSpecies], E[kMaxSpecies];
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
  for (int s = 0; s < S; ++s) {
    double a = 0, b = 0, cc = 0, d = 0;
    for (int i = 0; i < kNV; ++i) {
      const double v = (double)f[(size_t)(s * kNV + i) * I.ps + cell];
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
  // chemistry (Eqs.(1)-(2), one or several steps): extents, common clamp
  // factor, n* and T* from the energy balance
  double Tst = Tm, nst[kMaxSpecies];
  for (int s = 0; s < S; ++s) nst[s] = n[s];
  if (I.nreact > 0) {
    double xi[kMaxReact], scale = 1.0;
    for (int r = 0; r < I.nreact; ++r) {
      const double nF = fmax(n[I.rfuel[r]], 0.0), nO = fmax(n[I.roxid[r]], 0.0);
      xi[r] = I.rk[r] * nF * nO * exp(-I.rEa[r] / Tm) * sp[0].tau;
    }
    for (int s = 0; s < S; ++s) {
      double use = 0.0;
      for (int r = 0; r < I.nreact; ++r) use = fma(fmax(-I.ra[r][s], 0.0), xi[r], use);
      const double avail = fmax(n[s], 0.0);
      if (use > avail) scale = fmin(scale, avail / use);
    }
    double heat = 0.0, kns = 0.0;
    for (int r = 0; r < I.nreact; ++r) {
      xi[r] *= scale;
      heat = fma(I.rQ2[r], xi[r], heat);
      for (int s = 0; s < S; ++s) nst[s] = fma(I.ra[r][s], xi[r], nst[s]);
    }
    for (int s = 0; s < S; ++s) kns = fma(sp[s].K, nst[s], kns);
    Tst = fma(Tm, kn, heat) / kns;
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
    fhat(nst[s], ux, uy, Tst * sp[s].inv_m, g);
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

template <typename ST>
__global__ __launch_bounds__(256) void k_plain_eq(const InstDev *__restrict__ insts, int inst,
                                                  int in_idx) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  plain_feq_cell<ST>(I, fview<ST>(I, in_idx), plane, cell, (typename Stor<ST>::C *)I.scratch);
}

// Map a possibly-ghost index along one axis; walls reflect and flip.
__device__ __forceinline__ int map_axis(int j, int n, int bc, int &flips) {
  if (j >= 0 && j < n) return j;
  if (bc == BC_PERIODIC) {
    int q = j % n;
    return q < 0 ? q + n : q;
  }
  if (bc == BC_OUTFLOW) return j < 0 ? 0 : n - 1;
  int q = j % (2 * n);
  if (q < 0) q += 2 * n;
  if (q >= n) {
    flips ^= 1;
    return 2 * n - 1 - q;
  }
  return q;
}

template <typename ST>
__device__ __forceinline__ typename Stor<ST>::C plain_value(const InstDev &I, const FV<ST> &f,
                                                            size_t plane, int s, int i, int x,
                                                            int y) {
  int fx = 0, fy = 0;
  const int mx = map_axis(x, I.nx, I.bcx, fx), my = map_axis(y, I.ny, I.bcy, fy);
  int p = i;
  if (fx) p = I.sp[s].mirx[p];
  if (fy) p = I.sp[s].miry[p];
  return f[(size_t)(s * kNV + p) * I.ps + (size_t)my * I.nx + mx];
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

template <typename ST>
__device__ __forceinline__ void plain_update_cell(const InstDev *__restrict__ insts, int inst,
                                                  int in_idx, int fn_idx, int out_idx,
                                                  typename Stor<ST>::C alpha, int rkc, bool sr,
                                                  uint32_t step) {
  typedef typename Stor<ST>::C T;
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const int si = blockIdx.y, s = si / kNV, i = si % kNV;
  const int x = (int)(cell % I.nx), y = (int)(cell / I.nx);
  const FV<ST> f = fview<ST>(I, in_idx);
  const SpeciesDev &sp = I.sp[s];
  const double vx = sp.M[1 * kNV + i], vy = sp.M[2 * kNV + i];
  const T fc = f[(size_t)si * I.ps + cell];
  T C = T(0);
  if (vx != 0.0) {
    T w[5];
    for (int k = 0; k < 5; ++k) w[k] = plain_value<ST>(I, f, plane, s, i, x - 2 + k, y);
    const int sg = vx > 0 ? 1 : -1;
    const T fr = nnd_face<T>(w[1], w[2], w[3], w[4], sg, I.lim);
    const T fl = nnd_face<T>(w[0], w[1], w[2], w[3], sg, I.lim);
    C -= (T)(vx * I.dt / I.dx) * (fr - fl);
  }
  if (vy != 0.0) {
    T w[5];
    for (int k = 0; k < 5; ++k) w[k] = plain_value<ST>(I, f, plane, s, i, x, y - 2 + k);
    const int sg = vy > 0 ? 1 : -1;
    const T fr = nnd_face<T>(w[1], w[2], w[3], w[4], sg, I.lim);
    const T fl = nnd_face<T>(w[0], w[1], w[2], w[3], sg, I.lim);
    C -= (T)(vy * I.dt / I.dy) * (fr - fl);
  }
  const T feq = ((const T *)I.scratch)[(size_t)si * plane + cell];
  T res;
  if (sr) {   // stochastic rounding (see sr_add)
    T d = C + (T)sp.omega * (feq - fc);
    if (rkc) d = fma(alpha, (fview<ST>(I, fn_idx)[(size_t)si * I.ps + cell] - fc) - d, d);
    const uint32_t key = (uint32_t)cell * 0x9E3779B9u ^ (uint32_t)(si + 1) * 0x85EBCA6Bu ^
                         step * 0xC2B2AE35u ^ (uint32_t)__float_as_uint((float)fc);
    res = (T)sr_add((float)fc, (float)d, mix32(key));
  } else {
    res = fc + C + (T)sp.omega * (feq - fc);
    if (rkc) res = fma(alpha, fview<ST>(I, fn_idx)[(size_t)si * I.ps + cell] - res, res);
  }
  fview<ST>(I, out_idx).set((size_t)si * I.ps + cell, res);
}

template <typename ST>
__global__ __launch_bounds__(256) void k_plain_update(const InstDev *__restrict__ insts,
                                                      int inst, int in_idx, int fn_idx,
                                                      int out_idx, typename Stor<ST>::C alpha,
                                                      int rkc, int sr, uint32_t *ctr) {
  const bool kSR = std::is_same<ST, float>::value && sr;
  uint32_t step = 0;
  if (kSR) step = __hip_atomic_load(&ctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  plain_update_cell<ST>(insts, inst, in_idx, fn_idx, out_idx, alpha, rkc, kSR, step);
  if (kSR) advance_step_counter(ctr, step, gridDim.x * gridDim.y);
}

// ---------------------------------------------------------------------------
// Initialisation, diagnostics, conversion
// ---------------------------------------------------------------------------
// f := f^eq(n^s, u, T); fields = [n_sp (S planes), ux, uy, T] in FP64.
template <typename ST>
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
  const FV<ST> out = fview<ST>(I, out_idx);
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
    double fe[kNV];
    for (int r = 0; r < kNV; ++r) {
      double acc = 0.0;
      for (int k = 0; k < kNV; ++k) acc = fma(sp.Minv[r * kNV + k], h[k], acc);
      fe[r] = acc;
    }
    if (std::is_same<ST, float>::value && I.om) {
      float sv[kNV];
      uint16_t lo[4];
      om_pack(sp, om_rowref(I, s, (int)(cell / (size_t)I.nx)), fe, sv, I.ares ? lo : nullptr);
      for (int r = 0; r < kNV; ++r) ((float *)out.b)[(size_t)(s * kNV + r) * I.ps + cell] = sv[r];
      if (I.ares)
        for (int j = 0; j < 4; ++j) ares_ptr(I, out.b, s, j)[cell] = lo[j];
    } else {
      for (int r = 0; r < kNV; ++r) out.set((size_t)(s * kNV + r) * I.ps + cell, fe[r]);
    }
  }
}

// The 16 values f_i of species s at `cell`, widened to FP64 (reconstructed
// from OM storage when the buffers hold it).
template <typename ST>
__device__ __forceinline__ void cell_f(const InstDev &I, const FV<ST> &f, int s, size_t cell,
                                       double *out) {
  if constexpr (std::is_same<ST, float>::value) {
    if (I.om) {
      double sv[kNV];
      for (int i = 0; i < kNV; ++i) sv[i] = ((const float *)f.b)[(size_t)(s * kNV + i) * I.ps + cell];
      if (I.ares)
        for (int j = 0; j < 4; ++j) sv[j] += (double)bf16_value(ares_ptr(I, f.b, s, j)[cell]);
      om_unpack(I.sp[s], om_rowref(I, s, (int)(cell / (size_t)I.nx)), sv, out);
      return;
    }
  }
  for (int i = 0; i < kNV; ++i) out[i] = (double)f[(size_t)(s * kNV + i) * I.ps + cell];
}

// Per-cell species moments in FP64 (dense rows of M).
template <typename ST>
__device__ __forceinline__ void dense_moments(const InstDev &I, const FV<ST> &f, size_t plane,
                                              size_t cell, int s, double &n, double &jx,
                                              double &jy, double &E) {
  const SpeciesDev &sp = I.sp[s];
  double fv[kNV];
  cell_f<ST>(I, f, s, cell, fv);
  n = jx = jy = E = 0.0;
  for (int i = 0; i < kNV; ++i) {
    const double v = fv[i];
    n += v;
    jx = fma(v, sp.M[1 * kNV + i], jx);
    jy = fma(v, sp.M[2 * kNV + i], jy);
    E = fma(v, sp.M[3 * kNV + i], E);
  }
}

// dst = [rho_sp (S planes), ux, uy, T]
template <typename ST>
__global__ __launch_bounds__(256) void k_moments(const InstDev *__restrict__ insts, int inst,
                                                 int in_idx, double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const FV<ST> f = fview<ST>(I, in_idx);
  double rho = 0, px = 0, py = 0, e = 0, kn = 0;
  for (int s = 0; s < I.S; ++s) {
    double n, jx, jy, E;
    dense_moments<ST>(I, f, plane, cell, s, n, jx, jy, E);
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
template <typename ST>
__global__ __launch_bounds__(256) void k_noneq(const InstDev *__restrict__ insts, int inst,
                                               int in_idx, int which,
                                               double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const FV<ST> f = fview<ST>(I, in_idx);
  double rho = 0, px = 0, py = 0, e = 0, kn = 0, nw = 0;
  for (int s = 0; s < I.S; ++s) {
    double n, jx, jy, E;
    dense_moments<ST>(I, f, plane, cell, s, n, jx, jy, E);
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
  double dfv[kNV], fw[kNV];
  cell_f<ST>(I, f, which, cell, fw);
  for (int r = 0; r < kNV; ++r) {
    double acc = 0.0;
    for (int k = 0; k < kNV; ++k) acc = fma(sp.Minv[r * kNV + k], h[k], acc);
    dfv[r] = fw[r] - acc;
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
// Translational energies and energy fluxes of species `which` (the
// nonequilibrium measures section of the paper), 8 FP64 fields per cell:
//   1/2 M2xx(f), 1/2 M2yy(f), 1/2 M2xx(f^eq), 1/2 M2yy(f^eq),
//   1/2 M31x(f), 1/2 M31y(f), 1/2 M31x(f^eq), 1/2 M31y(f^eq),
// with M2aa(g) = m sum_i g_i v_ia^2 and M31a(g) = m sum_i g_i (v_i^2 + eta_i^2)
// v_ia; f^eq = f^eq(n^s, u, T) as for Delta.  Moments of f come from rows
// v_x^2, v_y^2, q v_x, q v_y of M; those of f^eq are the closed forms of
// fhat (M M^{-1} fhat = fhat).
template <typename ST>
__global__ __launch_bounds__(256) void k_energy(const InstDev *__restrict__ insts, int inst,
                                                int in_idx, int which,
                                                double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const FV<ST> f = fview<ST>(I, in_idx);
  double rho = 0, px = 0, py = 0, e = 0, kn = 0, nw = 0;
  for (int s = 0; s < I.S; ++s) {
    double n, jx, jy, E;
    dense_moments<ST>(I, f, plane, cell, s, n, jx, jy, E);
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
  const double th = Tm * sp.inv_m, u2 = ux * ux + uy * uy;
  const double e2 = (sp.K + 2.0) * th + u2;
  constexpr int rows[4] = {4, 6, 7, 8};  // v_x^2, v_y^2, q v_x, q v_y
  double mf[4], fw[kNV];
  cell_f<ST>(I, f, which, cell, fw);
  for (int r = 0; r < 4; ++r) {
    double acc = 0.0;
    for (int i = 0; i < kNV; ++i) acc = fma(sp.M[rows[r] * kNV + i], fw[i], acc);
    mf[r] = acc;
  }
  const double hm = 0.5 * sp.m;
  dst[0 * plane + cell] = hm * mf[0];
  dst[1 * plane + cell] = hm * mf[1];
  dst[2 * plane + cell] = hm * nw * (th + ux * ux);
  dst[3 * plane + cell] = hm * nw * (th + uy * uy);
  dst[4 * plane + cell] = hm * mf[2];
  dst[5 * plane + cell] = hm * mf[3];
  dst[6 * plane + cell] = hm * nw * ux * e2;
  dst[7 * plane + cell] = hm * nw * uy * e2;
}

constexpr int kTotThreads = 256;

// Partial totals per block: [block][S+3] = mass^s, Px, Py, E (unscaled).
template <typename ST>
__global__ __launch_bounds__(kTotThreads) void k_totals_partial(const InstDev *__restrict__ insts,
                                                                int inst, int in_idx,
                                                                double *__restrict__ part) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const FV<ST> f = fview<ST>(I, in_idx);
  const int S = I.S, nq = S + 3;
  double acc[kMaxSpecies + 3];
  for (int q = 0; q < nq; ++q) acc[q] = 0.0;
  for (size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cell < plane;
       cell += (size_t)gridDim.x * blockDim.x) {
    for (int s = 0; s < S; ++s) {
      double n, jx, jy, E;
      dense_moments<ST>(I, f, plane, cell, s, n, jx, jy, E);
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

// Deterministic per-block sums of nrows (<= kEnergyRows) FP64 fields of
// `cells` values each (fixed grid, fixed order), finished by k_totals_final.
constexpr int kEnergyRows = 8;
__global__ __launch_bounds__(kTotThreads) void k_rows_partial(const double *__restrict__ src,
                                                              int nrows, size_t cells,
                                                              double *__restrict__ part) {
  double acc[kEnergyRows];
  for (int r = 0; r < kEnergyRows; ++r) acc[r] = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
       c += (size_t)gridDim.x * blockDim.x)
    for (int r = 0; r < nrows; ++r) acc[r] += src[(size_t)r * cells + c];
  __shared__ double red[kTotThreads / kWave][kEnergyRows];
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  for (int r = 0; r < nrows; ++r) {
    const double v = wave_sum(acc[r]);
    if (l == 0) red[w][r] = v;
  }
  __syncthreads();
  if (threadIdx.x < nrows) {
    double s = 0.0;
    for (int k = 0; k < kTotThreads / kWave; ++k) s += red[k][threadIdx.x];
    part[(size_t)blockIdx.x * nrows + threadIdx.x] = s;
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

template <typename ST>
__global__ __launch_bounds__(256) void k_widen(const void *__restrict__ buf, size_t ntot,
                                               size_t first, double *__restrict__ dst,
                                               size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (double)FV<ST>(buf, ntot)[first + k];
}
template <typename ST>
__global__ __launch_bounds__(256) void k_narrow(const double *__restrict__ src,
                                                void *__restrict__ buf, size_t ntot,
                                                size_t first, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) FV<ST>(buf, ntot).set(first + k, (typename Stor<ST>::C)src[k]);
}

// OM storage transfers: plane i of species s of buffer b as FP64 (dst[cell]);
// the FP64 distribution staged as planes of stride I.ps, planes 0 .. 8S-1 in
// lo and the rest in hi, packed into buffer b; and an in-place change of
// representation of buffer b between FP32 f and OM storage (to_om).
__global__ __launch_bounds__(256) void k_widen_om(const InstDev *__restrict__ insts, int inst,
                                                  int b, int s, int i, double *__restrict__ dst) {
  const InstDev &I = insts[inst];
  const size_t cells = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= cells) return;
  double fv[kNV];
  cell_f<float>(I, fview<float>(I, b), s, cell, fv);
  dst[cell] = fv[i];
}
__global__ __launch_bounds__(256) void k_pack_om(const InstDev *__restrict__ insts, int inst,
                                                 const double *__restrict__ lo,
                                                 const double *__restrict__ hi, int b) {
  const InstDev &I = insts[inst];
  const size_t cells = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= cells) return;
  const int half = I.S * kNV / 2;
  float *out = (float *)I.buf[b];
  for (int s = 0; s < I.S; ++s) {
    double fv[kNV];
    float sv[kNV];
    for (int i = 0; i < kNV; ++i) {
      const int p = s * kNV + i;
      fv[i] = p < half ? lo[(size_t)p * I.ps + cell] : hi[(size_t)(p - half) * I.ps + cell];
    }
    uint16_t rl[4];
    om_pack(I.sp[s], om_rowref(I, s, (int)(cell / (size_t)I.nx)), fv, sv, I.ares ? rl : nullptr);
    for (int i = 0; i < kNV; ++i) out[(size_t)(s * kNV + i) * I.ps + cell] = sv[i];
    if (I.ares)
      for (int j = 0; j < 4; ++j) ares_ptr(I, out, s, j)[cell] = rl[j];
  }
}
// Changes the representation of buffer b in place, FP64 arithmetic per cell:
// from / to 0 f itself, 1 OM storage, 2 OM storage with A-block residuals.
__global__ __launch_bounds__(256) void k_convert_om(const InstDev *__restrict__ insts, int inst,
                                                    int b, int from, int to) {
  const InstDev &I = insts[inst];
  const size_t cells = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= cells) return;
  float *buf = (float *)I.buf[b];
  for (int s = 0; s < I.S; ++s) {
    double fv[kNV];
    const double *ref = om_rowref(I, s, (int)(cell / (size_t)I.nx));
    if (from == 0) {
      for (int i = 0; i < kNV; ++i) fv[i] = buf[(size_t)(s * kNV + i) * I.ps + cell];
    } else {
      double sv[kNV];
      for (int i = 0; i < kNV; ++i) sv[i] = buf[(size_t)(s * kNV + i) * I.ps + cell];
      if (from == 2)
        for (int j = 0; j < 4; ++j) sv[j] += (double)bf16_value(ares_ptr(I, buf, s, j)[cell]);
      om_unpack(I.sp[s], ref, sv, fv);
    }
    float out[kNV];
    uint16_t rl[4];
    if (to == 0) {
      for (int i = 0; i < kNV; ++i) out[i] = (float)fv[i];
    } else {
      om_pack(I.sp[s], ref, fv, out, to == 2 ? rl : nullptr);
    }
    for (int i = 0; i < kNV; ++i) buf[(size_t)(s * kNV + i) * I.ps + cell] = out[i];
    if (to == 2)
      for (int j = 0; j < 4; ++j) ares_ptr(I, buf, s, j)[cell] = rl[j];
  }
}

// Non-finite values, or a species density below -1e-12 of the local total.
template <typename ST>
__global__ __launch_bounds__(256) void k_check(const InstDev *__restrict__ insts, int inst,
                                               int in_idx, int *__restrict__ flag) {
  const InstDev &I = insts[inst];
  const size_t plane = (size_t)I.nx * I.ny;
  const size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= plane) return;
  const FV<ST> f = fview<ST>(I, in_idx);
  double tot = 0.0, nmin = 0.0;
  bool bad = false;
  for (int s = 0; s < I.S; ++s) {
    double n = 0.0, fv[kNV];
    cell_f<ST>(I, f, s, cell, fv);
    for (int i = 0; i < kNV; ++i) {
      const double v = fv[i];
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
  out[256 + l] = (int)shr1(v + 1.0f);
  out[320 + l] = (int)shl1(v + 1.0f);
  out[384 + l] = (int)shr1(d + 1.0);
  out[448 + l] = (int)shl1(d + 1.0);
  out[512 + l] = (int)row_bcast<4>(v);     // lane 16 (l / 16) + 4
  out[576 + l] = (int)quad_bcast<2>(v);    // lane 4 (l / 4) + 2
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
// Tile order: XCD-grouped (1, default) or plain dispatch order (0, for
// comparison; DBM_XCD_REMAP=0 in the environment), read once per process.
static int xcd_remap_flag() {
  static const int flag = [] {
    const char *e = getenv("DBM_XCD_REMAP");
    return (e && e[0] == '0') ? 0 : 1;
  }();
  return flag;
}

// One launch of the stage kernel: its arguments and the kernel variant.
struct FusedLaunch {
  const InstDev *insts;
  const Tile *tiles;
  int ntiles, grid, in_idx, fn_idx, out_idx, remap;
  double alpha, beta;
  bool split, pipe, sr, cw;  // split form, row pipeline, stochastic rounding, chain wavefront
  bool om;                   // FP32-bulk buffers in OM storage
  bool rowref;               // ... with references per grid row (else one per grid)
  bool ares;                 // ... with A-block residuals
  bool drain;                // ... every other row waits for its refill (k_fused_om)
  uint32_t *ctr;             // step counter of stochastic rounding
  hipStream_t st;
};

template <typename ST, int S, int LIM, bool RKC>
static hipError_t launch_fused_t(const FusedLaunch &a) {
  typedef typename Stor<ST>::C T;
  if constexpr (std::is_same<ST, float>::value) {
    if (a.om) {
      if (a.pipe || a.split) return hipErrorInvalidValue;
#define DBM_OM_LAUNCH3(R, C, Q, A)                                                              \
  hipLaunchKernelGGL((k_fused_om<S, LIM, RKC, R, C, Q, A>), dim3(a.grid),                       \
                     dim3(kWave * (S + (C ? 1 : 0))), 0, a.st, a.insts, a.tiles, a.ntiles,      \
                     a.in_idx, a.fn_idx, a.out_idx, (float)a.alpha, a.remap, a.ctr,          \
                     (int)a.drain)
#define DBM_OM_LAUNCH(R, C)                                                                     \
  do {                                                                                          \
    if (a.rowref) DBM_OM_LAUNCH3(R, C, true, false); else DBM_OM_LAUNCH3(R, C, false, false);  \
  } while (0)
#define DBM_OM_LAUNCH_AR(C)                                                                     \
  do {                                                                                          \
    if (a.rowref) DBM_OM_LAUNCH3(false, C, true, true);                                         \
    else DBM_OM_LAUNCH3(false, C, false, true);                                                 \
  } while (0)
      if (a.ares && a.sr) return hipErrorInvalidValue;
      if constexpr (S <= 3) {
        if (a.cw) {
          if (a.ares) DBM_OM_LAUNCH_AR(true);
          else if (a.sr) DBM_OM_LAUNCH(true, true);
          else DBM_OM_LAUNCH(false, true);
          return hipGetLastError();
        }
      }
      if (a.cw) return hipErrorInvalidValue;
      if (a.ares) DBM_OM_LAUNCH_AR(false);
      else if (a.sr) DBM_OM_LAUNCH(true, false);
      else DBM_OM_LAUNCH(false, false);
#undef DBM_OM_LAUNCH_AR
#undef DBM_OM_LAUNCH
#undef DBM_OM_LAUNCH3
      return hipGetLastError();
    }
  } else {
    if (a.om) return hipErrorInvalidValue;
  }
  if constexpr (!kSplitStore<ST>) {
    if (a.split) {
      hipLaunchKernelGGL((k_fused_split<ST, S, LIM, RKC>), dim3(a.grid), dim3(kWave * 2 * S), 0,
                         a.st, a.insts, a.tiles, a.ntiles, a.in_idx, a.fn_idx, a.out_idx,
                         (T)a.alpha, (T)a.beta, a.remap);
      return hipGetLastError();
    }
  }
#define DBM_FUSED_LAUNCH(P, R, C)                                                              \
  hipLaunchKernelGGL((k_fused_stage<ST, S, LIM, RKC, P, R, C>), dim3(a.grid),                   \
                     dim3(kWave * (S + (C ? 1 : 0))), 0, a.st, a.insts, a.tiles, a.ntiles,      \
                     a.in_idx, a.fn_idx, a.out_idx, (T)a.alpha, a.remap, a.ctr)
  if constexpr (S <= 3) {
    if (a.cw) {
      if (a.sr) DBM_FUSED_LAUNCH(false, true, true); else DBM_FUSED_LAUNCH(false, false, true);
      return hipGetLastError();
    }
  }
  if (a.cw) return hipErrorInvalidValue;
  if constexpr (std::is_same<ST, float>::value) {
    if (a.pipe) {
      if (a.sr) DBM_FUSED_LAUNCH(true, true, false); else DBM_FUSED_LAUNCH(true, false, false);
    } else {
      if (a.sr) DBM_FUSED_LAUNCH(false, true, false); else DBM_FUSED_LAUNCH(false, false, false);
    }
  } else {
    DBM_FUSED_LAUNCH(false, false, false);
  }
#undef DBM_FUSED_LAUNCH
  return hipGetLastError();
}

template <typename ST, int S, int LIM>
static hipError_t launch_fused_s(bool rkc, const FusedLaunch &a) {
  return rkc ? launch_fused_t<ST, S, LIM, true>(a) : launch_fused_t<ST, S, LIM, false>(a);
}

template <typename ST, int S>
static hipError_t launch_fused_l(int lim, bool rkc, const FusedLaunch &a) {
  return lim == DBM_LIM_MINMOD ? launch_fused_s<ST, S, DBM_LIM_MINMOD>(rkc, a)
                               : launch_fused_s<ST, S, DBM_LIM_NONE>(rkc, a);
}

template <typename ST>
static hipError_t launch_fused_p(int S, int lim, bool rkc, const FusedLaunch &a) {
  switch (S) {
    case 1: return launch_fused_l<ST, 1>(lim, rkc, a);
    case 2: return launch_fused_l<ST, 2>(lim, rkc, a);
    case 3: return launch_fused_l<ST, 3>(lim, rkc, a);
    case 4: return launch_fused_l<ST, 4>(lim, rkc, a);
    default: return hipErrorInvalidValue;
  }
}

// prec: DBM_FP64, DBM_FP32_BULK or DBM_FP32X (storage and arithmetic types).
// sr: stochastic rounding of the stores (FP32-bulk full form only).
// cw: chain wavefront (full form, S <= 3, no row pipeline).
// om: OM storage (FP32-bulk full form, no row pipeline): 1 one reference per
// grid, 2 references per row; ares: with A-block residuals (round to nearest
// only); drain: the OM kernel's form that waits for every other row's refill
// at once; ctr: step counter of stochastic rounding (two words of device
// memory).
hipError_t launch_fused(int prec, int S, int lim, bool rkc, bool split, bool pipe, bool sr,
                        bool cw, int om, bool ares, bool drain, uint32_t *ctr,
                        const InstDev *insts, const Tile *tiles, int ntiles, int grid,
                        int in_idx, int fn_idx, int out_idx, double alpha, double beta,
                        hipStream_t st) {
  if (prec == DBM_FP32X && split) return hipErrorInvalidValue;  // full form only
  if (sr && (prec != DBM_FP32_BULK || split || !ctr)) return hipErrorInvalidValue;
  if (cw && (split || pipe || S > 3)) return hipErrorInvalidValue;
  if (om && (prec != DBM_FP32_BULK || split || pipe)) return hipErrorInvalidValue;
  if (ares && (!om || sr)) return hipErrorInvalidValue;
  const FusedLaunch a{insts, tiles, ntiles, grid, in_idx, fn_idx, out_idx, xcd_remap_flag(),
                      alpha, beta, split, pipe, sr, cw, om != 0, om == 2, ares, drain, ctr, st};
  switch (prec) {
    case DBM_FP32_BULK: return launch_fused_p<float>(S, lim, rkc, a);
    case DBM_FP32X: return launch_fused_p<f32x>(S, lim, rkc, a);
    default: return launch_fused_p<double>(S, lim, rkc, a);
  }
}

template <typename ST, int S, int LIM, bool RKC>
constexpr auto k_fused_stage_np = k_fused_stage<ST, S, LIM, RKC, false, false, false>;
template <typename ST, int S, int LIM, bool RKC>
constexpr auto k_fused_stage_cw = k_fused_stage<ST, S, LIM, RKC, false, false, true>;

#define DBM_PICK1_CW(T, SS)                                                                     \
  fn = lim == DBM_LIM_MINMOD                                                                   \
           ? (rkc ? (const void *)k_fused_stage_cw<T, SS, DBM_LIM_MINMOD, true>                \
                  : (const void *)k_fused_stage_cw<T, SS, DBM_LIM_MINMOD, false>)              \
           : (rkc ? (const void *)k_fused_stage_cw<T, SS, DBM_LIM_NONE, true>                  \
                  : (const void *)k_fused_stage_cw<T, SS, DBM_LIM_NONE, false>)
#define DBM_PICK_CW(T)                                                                          \
  switch (S) { case 1: DBM_PICK1_CW(T, 1); break; case 2: DBM_PICK1_CW(T, 2); break;          \
               default: DBM_PICK1_CW(T, 3); break; }
// Workgroups of the stage kernel resident per CU (waves_per_cu), for the
// full form, the split form (split) or the chain-wavefront form (cw).
template <int S, int LIM, bool RKC, bool CW, bool AR>
constexpr auto k_fused_om_nr = k_fused_om<S, LIM, RKC, false, CW, true, AR>;

hipError_t fused_occupancy(int prec, int S, int lim, bool rkc, bool split, bool cw, bool om,
                           bool ares, int *waves_per_cu) {
  const void *fn = nullptr;
  if (om) {   // OM storage: FP32-bulk full form (ares: with A-block residuals)
    if (prec != DBM_FP32_BULK || split || (cw && S > 3)) {
      *waves_per_cu = 0;
      return hipSuccess;
    }
#define DBM_PICK_OM2(SS, C, A)                                                                  \
  fn = lim == DBM_LIM_MINMOD                                                                   \
           ? (rkc ? (const void *)k_fused_om_nr<SS, DBM_LIM_MINMOD, true, C, A>                \
                  : (const void *)k_fused_om_nr<SS, DBM_LIM_MINMOD, false, C, A>)              \
           : (rkc ? (const void *)k_fused_om_nr<SS, DBM_LIM_NONE, true, C, A>                  \
                  : (const void *)k_fused_om_nr<SS, DBM_LIM_NONE, false, C, A>)
#define DBM_PICK_OM(SS, C)                                                                      \
  do {                                                                                          \
    if (ares) DBM_PICK_OM2(SS, C, true); else DBM_PICK_OM2(SS, C, false);                       \
  } while (0)
    if (cw) {
      switch (S) { case 1: DBM_PICK_OM(1, true); break; case 2: DBM_PICK_OM(2, true); break;
                   default: DBM_PICK_OM(3, true); break; }
    } else {
      switch (S) { case 1: DBM_PICK_OM(1, false); break; case 2: DBM_PICK_OM(2, false); break;
                   case 3: DBM_PICK_OM(3, false); break; case 4: DBM_PICK_OM(4, false); break;
                   default: return hipErrorInvalidValue; }
    }
#undef DBM_PICK_OM
#undef DBM_PICK_OM2
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(waves_per_cu, fn,
                                                        kWave * (S + (cw ? 1 : 0)), 0);
  }
  if (prec == DBM_FP32X) split = false;  // full form only
  if (cw) {
    if (S > 3) {
      *waves_per_cu = 0;
      return hipSuccess;
    }
    if (prec == DBM_FP32_BULK) { DBM_PICK_CW(float); }
    else if (prec == DBM_FP32X) { DBM_PICK_CW(f32x); }
    else { DBM_PICK_CW(double); }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(waves_per_cu, fn, kWave * (S + 1), 0);
  }
#define DBM_PICK1(K, T, SS)                                                                     \
  fn = lim == DBM_LIM_MINMOD                                                                   \
           ? (rkc ? (const void *)K<T, SS, DBM_LIM_MINMOD, true>                               \
                  : (const void *)K<T, SS, DBM_LIM_MINMOD, false>)                             \
           : (rkc ? (const void *)K<T, SS, DBM_LIM_NONE, true>                                 \
                  : (const void *)K<T, SS, DBM_LIM_NONE, false>)
#define DBM_PICK(T, SS)                                                                         \
  if (split) { DBM_PICK1(k_fused_split, T, SS); } else { DBM_PICK1(k_fused_stage_np, T, SS); }
#define DBM_PICKX(SS) DBM_PICK1(k_fused_stage_np, f32x, SS)
  if (prec == DBM_FP32_BULK) {
    switch (S) { case 1: DBM_PICK(float, 1); break; case 2: DBM_PICK(float, 2); break;
                 case 3: DBM_PICK(float, 3); break; case 4: DBM_PICK(float, 4); break;
                 default: return hipErrorInvalidValue; }
  } else if (prec == DBM_FP32X) {
    switch (S) { case 1: DBM_PICKX(1); break; case 2: DBM_PICKX(2); break;
                 case 3: DBM_PICKX(3); break; case 4: DBM_PICKX(4); break;
                 default: return hipErrorInvalidValue; }
  } else {
    switch (S) { case 1: DBM_PICK(double, 1); break; case 2: DBM_PICK(double, 2); break;
                 case 3: DBM_PICK(double, 3); break; case 4: DBM_PICK(double, 4); break;
                 default: return hipErrorInvalidValue; }
  }
#undef DBM_PICK
#undef DBM_PICKX
#undef DBM_PICK1
#undef DBM_PICK1_CW
#undef DBM_PICK_CW
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(waves_per_cu, fn, kWave * S * (split ? 2 : 1),
                                                      0);
}

static inline unsigned blocks_for(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Launch kernel template K for the storage type of `prec`.
#define DBM_PREC_LAUNCH(prec, K, ...)                                                         \
  do {                                                                                        \
    switch (prec) {                                                                           \
      case DBM_FP32_BULK: hipLaunchKernelGGL((K<float>), __VA_ARGS__); break;                 \
      case DBM_FP32X: hipLaunchKernelGGL((K<f32x>), __VA_ARGS__); break;                      \
      default: hipLaunchKernelGGL((K<double>), __VA_ARGS__); break;                           \
    }                                                                                         \
  } while (0)

hipError_t launch_plain(int prec, const InstDev *insts, int inst, size_t cells, int S,
                        int in_idx, int fn_idx, int out_idx, double alpha, double beta, bool rkc,
                        bool sr, uint32_t *ctr, hipStream_t st) {
  if (sr && (prec != DBM_FP32_BULK || !ctr)) return hipErrorInvalidValue;
  (void)beta;  // alpha + beta = 1: the combine is res + alpha (f^n - res)
  const dim3 g1(blocks_for(cells, 256)), g2(blocks_for(cells, 256), (unsigned)(S * kNV));
  if (prec == DBM_FP32_BULK) {
    hipLaunchKernelGGL(k_plain_eq<float>, g1, dim3(256), 0, st, insts, inst, in_idx);
    hipLaunchKernelGGL(k_plain_update<float>, g2, dim3(256), 0, st, insts, inst, in_idx, fn_idx,
                       out_idx, (float)alpha, (int)rkc, (int)sr, ctr);
  } else if (prec == DBM_FP32X) {
    hipLaunchKernelGGL(k_plain_eq<f32x>, g1, dim3(256), 0, st, insts, inst, in_idx);
    hipLaunchKernelGGL(k_plain_update<f32x>, g2, dim3(256), 0, st, insts, inst, in_idx, fn_idx,
                       out_idx, alpha, (int)rkc, 0, ctr);
  } else {
    hipLaunchKernelGGL(k_plain_eq<double>, g1, dim3(256), 0, st, insts, inst, in_idx);
    hipLaunchKernelGGL(k_plain_update<double>, g2, dim3(256), 0, st, insts, inst, in_idx,
                       fn_idx, out_idx, alpha, (int)rkc, 0, ctr);
  }
  return hipGetLastError();
}

hipError_t launch_init(int prec, const InstDev *insts, int inst, size_t cells,
                       const double *fields, int out_idx, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_init_eq, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, fields, out_idx);
  return hipGetLastError();
}

hipError_t launch_moments(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                          double *dst, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_moments, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, dst);
  return hipGetLastError();
}

hipError_t launch_noneq(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int which, double *dst, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_noneq, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, which, dst);
  return hipGetLastError();
}

int totals_blocks() { return kTotBlocks; }
int energy_rows() { return kEnergyRows; }

hipError_t launch_energy(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                         int which, double *dst, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_energy, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, which, dst);
  return hipGetLastError();
}

hipError_t launch_rowsums(const double *src, int nrows, size_t cells, double area, double *part,
                          double *out, hipStream_t st) {
  if (nrows < 1 || nrows > kEnergyRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rows_partial, dim3(kTotBlocks), dim3(kTotThreads), 0, st, src, nrows,
                     cells, part);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, (const double *)part, kTotBlocks,
                     nrows, area, out);
  return hipGetLastError();
}

hipError_t launch_totals(int prec, const InstDev *insts, int inst, int in_idx, int nq,
                         double area, double *partials, double *out, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_totals_partial, dim3(kTotBlocks), dim3(kTotThreads), 0, st,
                       insts, inst, in_idx, partials);
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partials, kTotBlocks, nq, area,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch for the allocation-free totals entry point
// (dbm_noneq_totals_noalloc): the per-workgroup partial sums of
// k_totals_partial followed by the S+3 totals.  One copy per GPU, held until
// the process ends; host code addresses it only through the pointer
// hipGetSymbolAddress returns for the device (kept per device below).
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = 80 * 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Address of each device's `scratch`: looked up once per device, with that
// device current (the library's set-up, dbm_create), and kept for the
// entry point, which then only reads the table.
static std::mutex g_scratch_mu;
static void *g_scratch_addr[64] = {nullptr};

hipError_t static_scratch_init(int *device) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *device = dev;
  return hipSuccess;
}

void *static_scratch_get(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_addr[dev];
}

// Totals into the fixed scratch (partials, then the nq sums at `out`), or
// hipErrorInvalidValue when they do not fit.
hipError_t launch_totals_static(int prec, const InstDev *insts, int inst, int in_idx, int nq,
                                double area, void *scratch_ptr, double **out, hipStream_t st) {
  const size_t need = sizeof(double) * ((size_t)kTotBlocks * nq + nq);
  if (!scratch_ptr || nq < 1 || need > kStaticScratchBytes) return hipErrorInvalidValue;
  double *part = (double *)scratch_ptr;
  *out = part + (size_t)kTotBlocks * nq;
  return launch_totals(prec, insts, inst, in_idx, nq, area, part, *out, st);
}

// Values first .. first+n-1 of a buffer of ntot values <-> FP64.
hipError_t launch_widen(int prec, const void *buf, size_t ntot, size_t first, double *dst,
                        size_t n, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_widen, dim3(blocks_for(n, 256)), dim3(256), 0, st, buf, ntot, first,
                  dst, n);
  return hipGetLastError();
}

hipError_t launch_narrow(int prec, const double *src, void *buf, size_t ntot, size_t first,
                         size_t n, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_narrow, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, buf, ntot,
                  first, n);
  return hipGetLastError();
}

hipError_t launch_widen_om(const InstDev *insts, int inst, size_t cells, int b, int s, int i,
                           double *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_widen_om, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts, inst, b, s,
                     i, dst);
  return hipGetLastError();
}
hipError_t launch_pack_om(const InstDev *insts, int inst, size_t cells, const double *lo,
                          const double *hi, int b, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_om, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts, inst, lo, hi,
                     b);
  return hipGetLastError();
}
hipError_t launch_convert_om(const InstDev *insts, int inst, size_t cells, int b, int from, int to,
                             hipStream_t st) {
  if (from < 0 || from > 2 || to < 0 || to > 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_convert_om, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts, inst, b,
                     from, to);
  return hipGetLastError();
}

hipError_t launch_check(int prec, const InstDev *insts, int inst, size_t cells, int in_idx,
                        int *flag, hipStream_t st) {
  DBM_PREC_LAUNCH(prec, k_check, dim3(blocks_for(cells, 256)), dim3(256), 0, st, insts,
                       inst, in_idx, flag);
  return hipGetLastError();
}

// Streaming copy of n16 16-byte words (grid-stride, non-temporal stores):
// the achievable-bandwidth reference the stage kernel is compared with.
// Each thread keeps W words in flight per iteration (words i, i + stride,
// ..., so every load instruction of a wavefront reads 1 KiB contiguously).
template <int W>
__global__ __launch_bounds__(256) void k_copyw(const uint4 *__restrict__ src,
                                               uint4 *__restrict__ dst, size_t n16) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 *a = (const u32x4 *)src;
  u32x4 *b = (u32x4 *)dst;
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (W - 1) * stride < n16; i += W * stride) {
    u32x4 v[W];
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = a[i + w * stride];
#pragma unroll
    for (int w = 0; w < W; ++w) __builtin_nontemporal_store(v[w], &b[i + w * stride]);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(a[i], &b[i]);
}

hipError_t launch_copy16(const void *src, void *dst, size_t n16, int grid, int words,
                         hipStream_t st) {
  switch (words) {
    case 1: hipLaunchKernelGGL(k_copyw<1>, dim3(grid), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16); break;
    case 2: hipLaunchKernelGGL(k_copyw<2>, dim3(grid), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16); break;
    case 4: hipLaunchKernelGGL(k_copyw<4>, dim3(grid), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16); break;
    case 8: hipLaunchKernelGGL(k_copyw<8>, dim3(grid), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16); break;
    default: return hipErrorInvalidValue;
  }
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
