// Device arithmetic shared by the on-chip (resident) and streaming kernels of
// the Serial-EMD hot path: serialization and noise samples, block scans,
// reciprocals, run keys and knot emission on a blocked layout.  Included only
// by the library's .hip sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "semd_internal.h"

namespace semd {
namespace dev {

// A pointer into device memory, typed as the global address space.  Pointers
// read out of a descriptor in memory are otherwise generic, and accesses
// through them compile to flat instructions, which count against the LDS wait
// counter as well: every wait for an LDS result then also waits for the
// memory accesses in flight.  Through a global pointer they are global
// instructions, which also take a scalar base with a 32-bit lane offset.
template <class T>
using global_ptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ global_ptr<T> gmem(T* p) {
  return (global_ptr<T>)p;
}

constexpr int kWave = 64;
constexpr int kHalo = 32;    // rows a streaming solve window reaches beyond its block
constexpr int kRise = 1;
constexpr int kFall = 2;

// DPP controls: shift right (left) by n within each row of 16 lanes;
// broadcast lane 15 of each row to the next row; lane 31 to rows 2 and 3;
// shift the whole wave right (left) by one lane.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowShl = 0x100;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

// An int moved across lanes by a DPP control; lanes the control gives no
// source, and lanes of rows outside ROWS, get FILL.
template <int CTRL, int ROWS, int FILL = 0>
__device__ __forceinline__ int dpp_int(int x) {
  return __builtin_amdgcn_update_dpp(FILL, x, CTRL, ROWS, 0xf, false);
}

// The same for an int64 (each 32-bit half moved the same way; fill 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ int64_t dpp_i64(int64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROWS, 0xf, false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// A double of lane `src` (the same for the whole wave) to every lane.
__device__ __forceinline__ double lane_value(double x, int src) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, src);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A double moved across lanes by a DPP control (each 32-bit half moved the
// same way); lanes the control gives no source, and lanes of rows outside
// ROWS, get 0.0, or 1.0 when ONE is set.
template <int CTRL, int ROWS, bool ONE = false>
__device__ __forceinline__ double dpp_move(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(ONE ? 0x3ff00000 : 0, (int)(v >> 32), CTRL, ROWS,
                                             0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

// Direction of the step p -> q: rise, fall, or neither (equal or NaN).
__device__ __forceinline__ int step_kind(double p, double q) {
  return p < q ? kRise : (p > q ? kFall : 0);
}

// White noise sample k of a stream: Irwin-Hall sum of 12 uniforms on the
// 2^-53 grid, accumulated exactly as integers, centred, converted once.
__device__ __forceinline__ double noise_at(uint64_t key, int64_t k) {
  uint64_t acc = 0;
  const uint64_t c0 = 12ull * (uint64_t)k;
#pragma unroll
  for (int j = 0; j < 12; ++j) acc += splitmix64(key, c0 + (uint64_t)j + 1) >> 11;
  const int64_t c = (int64_t)acc - (int64_t)(6ull << 53);
  return (double)c * 0x1p-53;
}

// Serialized sample at row m of column i of T = [X ; E z] (Sec. 3.2).  Rows
// m >= M are the transition E: a_j X_A^f + a^f_j X_B^f with j = m - M + 1,
// a_j = j/(D+1); products and sum rounded separately (no contraction) so the
// value is the same on every device.
__device__ __forceinline__ double serial_at(const double* __restrict__ X, int64_t M, int32_t D,
                                            int64_t i, int64_t m) {
  if (m < M) return X[i * M + m];
  const int64_t j = m - M + 1;
  const double den = (double)(D + 1);
  const double a = (double)j / den;
  const double af = (double)(D + 1 - j) / den;
  const double xa = X[(i + 1) * M + (D - j)];
  const double xb = X[i * M + (M - j)];
  return __dadd_rn(__dmul_rn(xa, a), __dmul_rn(xb, af));
}

__host__ __device__ constexpr int knot_cap(int L) {
  // at most ceil((L-2)/2) extrema of one kind, plus 4 mirrored knots
  return (L > 1 ? (L - 1) / 2 : 0) + 4;
}

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// Block-wide exclusive prefix sum of one int per thread (a DPP scan within
// each wave, then the wave totals through LDS).  Contains one barrier.
template <int NW>
__device__ __forceinline__ int block_excl_sum(int v, int* wagg, int lane, int wid, int& total) {
  int inc = v;
  inc += dpp_int<kDppRowShr + 1, 0xf>(inc);
  inc += dpp_int<kDppRowShr + 2, 0xf>(inc);
  inc += dpp_int<kDppRowShr + 4, 0xf>(inc);
  inc += dpp_int<kDppRowShr + 8, 0xf>(inc);
  inc += dpp_int<kDppRowBcast15, 0xa>(inc);
  inc += dpp_int<kDppRowBcast31, 0xc>(inc);
  if (lane == kWave - 1) wagg[wid] = inc;
  __syncthreads();
  // the wave totals, one per lane of the first row, scanned the same way
  static_assert(NW <= 16, "wave totals fit one row of lanes");
  int w = lane < NW ? wagg[lane] : 0;
  w += dpp_int<kDppRowShr + 1, 0xf>(w);
  w += dpp_int<kDppRowShr + 2, 0xf>(w);
  w += dpp_int<kDppRowShr + 4, 0xf>(w);
  w += dpp_int<kDppRowShr + 8, 0xf>(w);
  const int uw = __builtin_amdgcn_readfirstlane(wid);
  total = __builtin_amdgcn_readlane(w, NW - 1);
  const int before = uw > 0 ? __builtin_amdgcn_readlane(w, uw - 1) : 0;
  return before + inc - v;
}

// Block-wide sums of two doubles per thread (a DPP scan within each wave,
// whose last lane holds the wave's sums, then the wave sums through LDS,
// 2*NW doubles, added by one wave-wide scan whose result every thread
// reads, so all get the same totals).  Contains one barrier; wsum must not
// be in use.
template <int NW>
__device__ __forceinline__ void block_sum2(double a, double b, double* wsum, int lane, int wid,
                                           double& ta, double& tb) {
#define SEMD_SUM_STEP(ctrl, rows)            \
  a += dpp_move<ctrl, rows>(a);              \
  b += dpp_move<ctrl, rows>(b);
  SEMD_SUM_STEP(kDppRowShr + 1, 0xf)
  SEMD_SUM_STEP(kDppRowShr + 2, 0xf)
  SEMD_SUM_STEP(kDppRowShr + 4, 0xf)
  SEMD_SUM_STEP(kDppRowShr + 8, 0xf)
  SEMD_SUM_STEP(kDppRowBcast15, 0xa)
  SEMD_SUM_STEP(kDppRowBcast31, 0xc)
#undef SEMD_SUM_STEP
  if (lane == kWave - 1) {
    wsum[2 * wid] = a;
    wsum[2 * wid + 1] = b;
  }
  __syncthreads();
  // the wave sums, one pair per lane of the first row, added by DPP shifts
  static_assert(NW <= 16, "wave sums fit one row of lanes");
  double sa = lane < NW ? wsum[2 * lane] : 0.0, sb = lane < NW ? wsum[2 * lane + 1] : 0.0;
  sa += dpp_move<kDppRowShr + 1, 0xf>(sa);
  sb += dpp_move<kDppRowShr + 1, 0xf>(sb);
  sa += dpp_move<kDppRowShr + 2, 0xf>(sa);
  sb += dpp_move<kDppRowShr + 2, 0xf>(sb);
  sa += dpp_move<kDppRowShr + 4, 0xf>(sa);
  sb += dpp_move<kDppRowShr + 4, 0xf>(sb);
  sa += dpp_move<kDppRowShr + 8, 0xf>(sa);
  sb += dpp_move<kDppRowShr + 8, 0xf>(sb);
  ta = lane_value(sa, NW - 1);
  tb = lane_value(sb, NW - 1);
}

// 1/x for positive normal x: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r); within an ulp of 1/x.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Extrema (Sec. 2.1 Step 1) on a blocked layout
// ---------------------------------------------------------------------------

// Kind code of a run that started before the block and whose start is not
// known yet (its first sample is the block's first).
constexpr int kCont = 3;

// Write this thread's knots of one kind (bits) at global ranks first.. among
// n, plus the mirrored end knots: the knot list is
//   [-k_P', ..., -k_1, k_1, ..., k_n, 2(L-1)-k_n, ..., 2(L-1)-k_{n-P'+1}],
// P' = min(2, n), mirrored knots carrying their source's value.
// Writes at index limit or beyond are dropped (they cannot happen when the
// counts and the flags agree).
template <int C, typename T>
__device__ __forceinline__ void emit_knots(const double (&h)[C], unsigned bits, int carry,
                                           int base, int nv, int L, int first, int n, T* kt,
                                           double* ky, int limit) {
  if (bits == 0u || n < 1) return;
  const int Pp = n < 2 ? n : 2;
  const int hi = 2 * (L - 1);
  int g = first;
  int start = carry >> 2;
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    if (c < nv) {
      const int k = base + c;
      if (c > 0 && h[c - 1] != h[c]) start = k;
      if ((bits >> c) & 1u) {
        const int mid = (start + k) >> 1;
        const double y = h[c];
        if (Pp + g < limit) { kt[Pp + g] = (T)mid; ky[Pp + g] = y; }
        if (g == 0) { kt[Pp - 1] = (T)(-mid); ky[Pp - 1] = y; }
        if (g == 1 && Pp == 2) { kt[0] = (T)(-mid); ky[0] = y; }
        if (g == n - 1 && Pp + n < limit) { kt[Pp + n] = (T)(hi - mid); ky[Pp + n] = y; }
        if (g == n - 2 && Pp == 2 && Pp + n + 1 < limit) {
          kt[Pp + n + 1] = (T)(hi - mid);
          ky[Pp + n + 1] = y;
        }
        ++g;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Scans for the natural-spline solve (Sec. 2.1 Step 2).  Forward
// elimination of the tridiagonal system in homogeneous form, one row being
// the linear map  Q' = b Q - a P,  P' = c Q,  D' = r Q - a D  (so that
// c' = P/Q and d' = D/Q), composes associatively and is scanned as 3x3 maps
// of the shape [[A, 0], [v^T, s]]; back-substitution M = d' - c' M_next is
// scanned as affine maps from the end.  Powers of two rescale the
// homogeneous quantities exactly, changing no ratio.
// ---------------------------------------------------------------------------

// Doubles per wave aggregate of the forward scan in LDS (7 used, padded to
// 16-byte multiples so an aggregate is read with 128-bit loads).
constexpr int kFwdStride = 8;

// One forward map, x -> (a00 Q + a01 P, a10 Q + a11 P, v0 Q + v1 P + s D).
struct FwdMap {
  double a00, a01, a10, a11, v0, v1, s;
};

__device__ __forceinline__ FwdMap fwd_identity() { return {1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0}; }

// X after Y.
__device__ __forceinline__ FwdMap fwd_compose(const FwdMap& X, const FwdMap& Y) {
  FwdMap Z;
  Z.a00 = fma(X.a00, Y.a00, X.a01 * Y.a10);
  Z.a01 = fma(X.a00, Y.a01, X.a01 * Y.a11);
  Z.a10 = fma(X.a10, Y.a00, X.a11 * Y.a10);
  Z.a11 = fma(X.a10, Y.a01, X.a11 * Y.a11);
  Z.v0 = fma(X.v0, Y.a00, fma(X.v1, Y.a10, X.s * Y.v0));
  Z.v1 = fma(X.v0, Y.a01, fma(X.v1, Y.a11, X.s * Y.v1));
  Z.s = X.s * Y.s;
  return Z;
}

// Row k's map after X: a cheaper compose for the sparse row map.
__device__ __forceinline__ FwdMap fwd_row_after(double a, double b, double c, double r,
                                                const FwdMap& X) {
  FwdMap Z;
  Z.a00 = fma(b, X.a00, -a * X.a10);
  Z.a01 = fma(b, X.a01, -a * X.a11);
  Z.a10 = c * X.a00;
  Z.a11 = c * X.a01;
  Z.v0 = fma(r, X.a00, -a * X.v0);
  Z.v1 = fma(r, X.a01, -a * X.v1);
  Z.s = -a * X.s;
  return Z;
}

// Exact rescaling by a power of two bringing |A| near 1.
__device__ __forceinline__ void fwd_normalize(FwdMap& X) {
  const int ex = __builtin_amdgcn_frexp_exp(fabs(X.a00) + fabs(X.a01) + fabs(X.a10) +
                                            fabs(X.a11));
  X.a00 = __builtin_amdgcn_ldexp(X.a00, -ex);
  X.a01 = __builtin_amdgcn_ldexp(X.a01, -ex);
  X.a10 = __builtin_amdgcn_ldexp(X.a10, -ex);
  X.a11 = __builtin_amdgcn_ldexp(X.a11, -ex);
  X.v0 = __builtin_amdgcn_ldexp(X.v0, -ex);
  X.v1 = __builtin_amdgcn_ldexp(X.v1, -ex);
  X.s = __builtin_amdgcn_ldexp(X.s, -ex);
}

__device__ __forceinline__ void fwd_apply(const FwdMap& X, double& Q, double& P, double& D) {
  const double q = fma(X.a00, Q, X.a01 * P);
  const double p = fma(X.a10, Q, X.a11 * P);
  D = fma(X.v0, Q, fma(X.v1, P, X.s * D));
  Q = q;
  P = p;
}

__device__ __forceinline__ void vec_normalize(double& Q, double& P, double& D) {
  const int ex = __builtin_amdgcn_frexp_exp(Q);  // Q > 0
  Q = __builtin_amdgcn_ldexp(Q, -ex);
  P = __builtin_amdgcn_ldexp(P, -ex);
  D = __builtin_amdgcn_ldexp(D, -ex);
}

// A map moved across lanes; lanes without a source get the identity, which
// composes and applies exactly (no rounding), so that the scans need no
// per-lane selection.
template <int CTRL, int ROWS>
__device__ __forceinline__ FwdMap fwd_dpp(const FwdMap& X) {
  return {dpp_move<CTRL, ROWS, true>(X.a00), dpp_move<CTRL, ROWS>(X.a01),
          dpp_move<CTRL, ROWS>(X.a10),       dpp_move<CTRL, ROWS, true>(X.a11),
          dpp_move<CTRL, ROWS>(X.v0),        dpp_move<CTRL, ROWS>(X.v1),
          dpp_move<CTRL, ROWS, true>(X.s)};
}


// Inclusive scan of the maps over the lanes of a wave (lane l gets the
// composition of lanes 0..l, later after earlier): Kogge-Stone within each
// row of 16 lanes, then the row totals broadcast down the wave.
__device__ __forceinline__ FwdMap fwd_wave_scan(FwdMap G) {
  // (the first n lanes of each row under a shift by n, and the rows a
  // broadcast skips, compose with the identity)
  G = fwd_compose(G, fwd_dpp<kDppRowShr + 1, 0xf>(G));
  G = fwd_compose(G, fwd_dpp<kDppRowShr + 2, 0xf>(G));
  G = fwd_compose(G, fwd_dpp<kDppRowShr + 4, 0xf>(G));
  G = fwd_compose(G, fwd_dpp<kDppRowShr + 8, 0xf>(G));
  G = fwd_compose(G, fwd_dpp<kDppRowBcast15, 0xa>(G));
  G = fwd_compose(G, fwd_dpp<kDppRowBcast31, 0xc>(G));
  return G;
}

// The state (Q, P, D) entering wave wid: the aggregates of waves 0..wid-1
// applied to (1, 0, 0) in order.
__device__ __forceinline__ void fwd_enter(const double* fwd_lds, int wid, double& Q, double& P,
                                          double& D) {
  Q = 1.0;
  P = 0.0;
  D = 0.0;
  // (the wave index is the same in every lane: a scalar loop)
  const int uw = __builtin_amdgcn_readfirstlane(wid);
  for (int w = 0; w < uw; ++w) {
    const double2* o = reinterpret_cast<const double2*>(fwd_lds + kFwdStride * w);
    const double2 x0 = o[0], x1 = o[1], x2 = o[2], x3 = o[3];
    const FwdMap X = {x0.x, x0.y, x1.x, x1.y, x2.x, x2.y, x3.x};
    fwd_apply(X, Q, P, D);
    vec_normalize(Q, P, D);
  }
}

// Suffix scan of back-substitution maps x -> al + be x over the lanes of a
// wave (lane l gets lanes l..63 composed, l's map applied last): within
// each row of 16 lanes by DPP shifts, then the later rows' totals.  With
// kFill the last n lanes of each row under a shift by n compose with the
// identity x -> 0 + 1 x (exact) instead of keeping their maps by a select;
// the two give the same values and differ only in register demand.
template <bool kFill = true>
__device__ __forceinline__ void bwd_wave_scan(double& al, double& be, int lane) {
#define SEMD_BWD_STEP(n)                                                        \
  {                                                                             \
    const double a2 = dpp_move<kDppRowShl + n, 0xf>(al);                        \
    const double b2 = dpp_move<kDppRowShl + n, 0xf, kFill>(be);                 \
    if (kFill || (lane & 15) + n < 16) {                                        \
      al = fma(be, a2, al);                                                     \
      be = be * b2;                                                             \
    }                                                                           \
  }
  SEMD_BWD_STEP(1)
  SEMD_BWD_STEP(2)
  SEMD_BWD_STEP(4)
  SEMD_BWD_STEP(8)
#undef SEMD_BWD_STEP
  const int row = lane >> 4;
  if (kFill) {
    // the totals of rows 1..3 (their lane 0) read out and composed once:
    // after row 2 comes T3, after row 1 T2 T3, after row 0 T1 T2 T3
    const double a1 = lane_value(al, 16), b1 = lane_value(be, 16);
    const double a2 = lane_value(al, 32), b2 = lane_value(be, 32);
    const double a3 = lane_value(al, 48), b3 = lane_value(be, 48);
    const double s1a = fma(b2, a3, a2), s1b = b2 * b3;
    const double s0a = fma(b1, s1a, a1), s0b = b1 * s1b;
    const double sa = row == 0 ? s0a : (row == 1 ? s1a : (row == 2 ? a3 : 0.0));
    const double sb = row == 0 ? s0b : (row == 1 ? s1b : (row == 2 ? b3 : 1.0));
    al = fma(be, sa, al);
    be = be * sb;
    return;
  }
  // rows 0..2 take row r+1's total (its lane 0), then rows 0..1 row r+2's
  {
    const int src = min(row + 1, 3) << 4;
    const double a2 = __shfl(al, src, kWave), b2 = __shfl(be, src, kWave);
    if (row < 3) { al = fma(be, a2, al); be = be * b2; }
  }
  {
    const int src = min(row + 2, 3) << 4;
    const double a2 = __shfl(al, src, kWave), b2 = __shfl(be, src, kWave);
    if (row < 2) { al = fma(be, a2, al); be = be * b2; }
  }
}

// M at the first row after wave wid: the later waves' maps applied to 0.
__device__ __forceinline__ double bwd_after(const double* bwd_lds, int wid, int wact) {
  double Mn = 0.0;
  // (wave index and count are the same in every lane: a scalar loop)
  const int uw = __builtin_amdgcn_readfirstlane(wid), ua = __builtin_amdgcn_readfirstlane(wact);
  for (int w = ua - 1; w > uw; --w) Mn = fma(bwd_lds[2 * w + 1], Mn, bwd_lds[2 * w]);
  return Mn;
}

}  // namespace dev
}  // namespace semd
