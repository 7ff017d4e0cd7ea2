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

constexpr int kWave = 64;
constexpr int kChunk = 8;    // interior spline unknowns solved per thread
constexpr int kHalo = 32;    // knots swept on each side beyond a chunk
constexpr int kRise = 1;
constexpr int kFall = 2;

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

// Block-wide exclusive prefix sum of one int per thread (wave shuffles, then
// the wave totals through LDS).  Contains one barrier.
template <int NW>
__device__ __forceinline__ int block_excl_sum(int v, int* wagg, int lane, int wid, int& total) {
  int inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int u = __shfl_up(inc, d, kWave);
    if (lane >= d) inc += u;
  }
  if (lane == kWave - 1) wagg[wid] = inc;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int a = wagg[w];
    before += (w < wid) ? a : 0;
    tot += a;
  }
  total = tot;
  return before + inc - v;
}

// Block-wide sums of two doubles per thread (wave shuffles, then the wave
// sums through LDS, 2*NW doubles, added in wave order so every thread gets
// the same totals).  Contains one barrier; wsum must not be in use.
template <int NW>
__device__ __forceinline__ void block_sum2(double a, double b, double* wsum, int lane, int wid,
                                           double& ta, double& tb) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    a += __shfl_xor(a, d, kWave);
    b += __shfl_xor(b, d, kWave);
  }
  if (lane == 0) {
    wsum[2 * wid] = a;
    wsum[2 * wid + 1] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sa += wsum[2 * w];
    sb += wsum[2 * w + 1];
  }
  ta = sa;
  tb = sb;
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

}  // namespace dev
}  // namespace semd
