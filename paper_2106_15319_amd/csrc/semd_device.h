// Device arithmetic shared by the on-chip (resident) and streaming kernels of
// the Serial-EMD hot path: serialization and noise samples, extremum
// detection and knot emission on a blocked layout, the natural-spline solve
// and the spline walker.  Included only by the library's .hip sources.
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

// A block holds samples a .. a+n-1 of a signal of length L; thread t owns
// the C samples starting at a + t*C, in registers h[].  Each thread
// publishes its first and last sample and the key (4*index + step kind) of
// the last run start strictly inside its samples; after one barrier every
// thread knows its neighbours and the start of the run its first sample
// belongs to (first_key is that key for the block's first sample; next_halo
// is sample a+n).  A sample k <= L-2 where the run ends (h[k+1] != h[k])
// closes a maximum if the run was entered rising and is left falling
// (minimum: the reverse), at the floor-middle of the run.  Runs that start at
// sample 0 have step kind 0 and never yield an extremum; the run that ends at
// L-1 is never closed.  A run of kind kCont yields no extremum either; if it
// ends inside the block, the direction it is left in (kFall or kRise) is
// written to *cont_exit.  *last_key (if given) receives the key of the run
// holding the thread's last sample, -1 for a thread without samples.
template <int NT, int C>
__device__ __forceinline__ void detect_extrema(const double (&h)[C], int a, int n, int L, int tid,
                                               int first_key, double next_halo,
                                               double* pub_first, double* pub_last,
                                               int* pub_key, int& carry, unsigned& maxbits,
                                               unsigned& minbits, int& cmax, int& cmin,
                                               int* cont_exit, int* last_key) {
  const int lb = tid * C;
  const int base = a + lb;
  const int nv = max(0, min(C, n - lb));
  if (nv > 0) {
    double last = h[0];
    int key = -1;
#pragma unroll
    for (int c = 1; c < C; ++c) {
      if (c < nv) {
        last = h[c];
        if (h[c - 1] != h[c]) key = (base + c) * 4 + step_kind(h[c - 1], h[c]);
      }
    }
    pub_first[tid] = h[0];
    pub_last[tid] = last;
    pub_key[tid] = key;
  }
  __syncthreads();
  double next = 0.0;
  if (nv == C && base + C < L) next = (lb + C < n) ? pub_first[tid + 1] : next_halo;
  carry = first_key;
  if (nv > 0 && tid > 0) {
    const double prev = pub_last[tid - 1];
    if (prev != h[0]) {
      carry = base * 4 + step_kind(prev, h[0]);
    } else {
      // the run continues from an earlier thread: walk back to its start
      int tau = tid - 1;
      for (;;) {
        const int kk = pub_key[tau];
        if (kk >= 0) { carry = kk; break; }
        if (tau == 0) { carry = first_key; break; }
        const double pl = pub_last[tau - 1], pf = pub_first[tau];
        if (pl != pf) { carry = (a + tau * C) * 4 + step_kind(pl, pf); break; }
        --tau;
      }
    }
  }
  maxbits = 0u;
  minbits = 0u;
  cmax = 0;
  cmin = 0;
  int cur = carry;
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    if (c < nv) {
      const int k = base + c;
      if (c > 0 && h[c - 1] != h[c]) cur = k * 4 + step_kind(h[c - 1], h[c]);
      if (k <= L - 2) {
        const double hn = (c + 1 < nv) ? h[c + 1 < C ? c + 1 : C - 1] : next;
        if (hn != h[c]) {
          const int kind = cur & 3;
          if (kind == kRise && hn < h[c]) { maxbits |= 1u << c; ++cmax; }
          else if (kind == kFall && hn > h[c]) { minbits |= 1u << c; ++cmin; }
          else if (kind == kCont && cont_exit) *cont_exit = hn < h[c] ? kFall : kRise;
        }
      }
    }
  }
  if (last_key) *last_key = nv > 0 ? cur : -1;
}

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
// Natural cubic spline (Sec. 2.1 Step 2): second derivatives
// ---------------------------------------------------------------------------

// Knots t_0 < ... < t_{n-1} (n >= 3), M_0 = M_{n-1} = 0 and for 1 <= j <= n-2
//   g_{j-1} M_{j-1} + 2 (g_{j-1} + g_j) M_j + g_j M_{j+1}
//       = 6 ((y_{j+1} - y_j)/g_j - (y_j - y_{j-1})/g_{j-1}).
// The interior unknowns are cut into chunks of kChunk; one thread solves a
// chunk by a forward Thomas sweep that starts kHalo rows before the chunk and
// a backward sweep that starts kHalo rows after it (run interleaved, they are
// independent), joined at the chunk's last row, then back-substitutes.
// Windows that reach the true ends of the system are exact; elsewhere the
// dropped coupling beyond the window is damped by at least (2-sqrt 3)^kHalo:
// the matrix is symmetric and diagonally dominant by a factor 2 in every row,
// so its Jacobi-scaled form has condition number at most 3 and an inverse
// whose entries decay geometrically with that ratio.
// kt and ky may hold only a window of the knots: element j sits at j - koff.
template <typename T>
__device__ __forceinline__ void solve_chunk(const T* __restrict__ kt,
                                            const double* __restrict__ ky, int koff,
                                            double* __restrict__ km, int n, int ch) {
  const int s = 1 + ch * kChunk;
  const int e = min(s + kChunk - 1, n - 2);
  const int ws = max(1, s - kHalo);
  const int we = min(n - 2, e + kHalo);

  // forward sweep, positioned at row ws with row ws-1 standing in for the
  // coupling it drops (cp = dp = 0)
  double ftp = (double)kt[ws - 1 - koff], ft = (double)kt[ws - koff];
  double fy = ky[ws - koff];
  double fsp = (fy - ky[ws - 1 - koff]) * recip(ft - ftp);
  double cp = 0.0, dp = 0.0;
  // backward sweep, positioned at row we with row we+1 standing in likewise
  double btn = (double)kt[we + 1 - koff], bt = (double)kt[we - koff];
  double by = ky[we - koff];
  double bsn = (ky[we + 1 - koff] - by) * recip(btn - bt);
  double aa = 0.0, dd = 0.0;

  const int nf = s - ws;                    // forward halo rows ws .. s-1
  const int nb = (e < n - 2) ? we - e : 0;  // backward rows we .. e+1
  const int steps = max(nf, nb);
  for (int i = 0; i < steps; ++i) {
    if (i < nf) {
      const int j = ws + i;
      const double tn = (double)kt[j + 1 - koff], yn = ky[j + 1 - koff];
      const double g0 = ft - ftp, g1 = tn - ft;
      const double sn = (yn - fy) * recip(g1);
      const double rhs = 6.0 * (sn - fsp);
      const double inv = recip(fma(-g0, cp, 2.0 * (g0 + g1)));
      cp = g1 * inv;
      dp = fma(-g0, dp, rhs) * inv;
      ftp = ft; ft = tn; fy = yn; fsp = sn;
    }
    if (i < nb) {
      const int j = we - i;
      const double tp = (double)kt[j - 1 - koff], yp = ky[j - 1 - koff];
      const double g1 = btn - bt, g0 = bt - tp;
      const double sp = (by - yp) * recip(g0);
      const double rhs = 6.0 * (bsn - sp);
      const double inv = recip(fma(-g1, aa, 2.0 * (g0 + g1)));
      aa = g0 * inv;
      dd = fma(-g1, dd, rhs) * inv;
      btn = bt; bt = tp; by = yp; bsn = sp;
    }
  }
  double cpa[kChunk], dpa[kChunk];
#pragma unroll
  for (int q = 0; q < kChunk; ++q) {
    cpa[q] = 0.0;
    dpa[q] = 0.0;
    if (s + q <= e) {
      const int j = s + q;
      const double tn = (double)kt[j + 1 - koff], yn = ky[j + 1 - koff];
      const double g0 = ft - ftp, g1 = tn - ft;
      const double sn = (yn - fy) * recip(g1);
      const double rhs = 6.0 * (sn - fsp);
      const double inv = recip(fma(-g0, cp, 2.0 * (g0 + g1)));
      cp = g1 * inv;
      dp = fma(-g0, dp, rhs) * inv;
      cpa[q] = cp;
      dpa[q] = dp;
      ftp = ft; ft = tn; fy = yn; fsp = sn;
    }
  }
  // M_e = dp - cp M_{e+1} with M_{e+1} = dd - aa M_e from the right, or
  // M_e = dp on the last row (M_{n-1} = 0)
  const double Me = (e < n - 2) ? fma(-cp, dd, dp) * recip(fma(-cp, aa, 1.0)) : dp;
  km[e] = Me;
  double Mn = Me;
#pragma unroll
  for (int q = kChunk - 1; q >= 0; --q) {
    if (s + q < e) {
      Mn = fma(-cpa[q], Mn, dpa[q]);
      km[s + q] = Mn;
    }
  }
}

// Second derivatives of up to two independent knot systems held in LDS: n1
// knots at offset 0 and n2 knots at offset o2 (n = 0: no system).  Their
// chunks are spread over the workgroup's threads.
template <int NT, typename T>
__device__ void spline_second_derivs(const T* __restrict__ kt,
                                     const double* __restrict__ ky, double* __restrict__ km,
                                     int n1, int o2, int n2, int tid) {
  const int c1 = n1 >= 3 ? (n1 - 2 + kChunk - 1) / kChunk : 0;
  const int c2 = n2 >= 3 ? (n2 - 2 + kChunk - 1) / kChunk : 0;
  for (int ch = tid; ch < c1 + c2; ch += NT) {
    const bool second = ch >= c1;
    const int o = second ? o2 : 0;
    solve_chunk(kt + o, ky + o, 0, km + o, second ? n2 : n1, second ? ch - c1 : ch);
  }
  if (tid == 0) {
    if (n1 >= 3) { km[0] = 0.0; km[n1 - 1] = 0.0; }
    if (n2 >= 3) { km[o2] = 0.0; km[o2 + n2 - 1] = 0.0; }
  }
}

// ---------------------------------------------------------------------------
// Spline evaluation: one walker per envelope and thread
// ---------------------------------------------------------------------------

// The current segment [t0, t1) of a walker, in the form
//   S(k) = a3 A^3 + b3 B^3 + p A + q B,  A = t1 - k,  B = k - t0,
// with a3 = M_j/(6g), b3 = M_{j+1}/(6g), p = (y_j - M_j g^2/6)/g and
// q = (y_{j+1} - M_{j+1} g^2/6)/g (g = t1 - t0): the textbook form of the
// natural spline on a segment, with its divisions done once per segment.
struct Seg {
  int j;
  double t0, t1;
  double a3, b3, p, q;
};

template <typename T>
__device__ __forceinline__ void seg_load(Seg& s, const T* __restrict__ kt,
                                         const double* __restrict__ ky,
                                         const double* __restrict__ km, int j) {
  s.j = j;
  s.t0 = (double)kt[j];
  s.t1 = (double)kt[j + 1];
  const double y0 = ky[j], m0 = km[j], y1 = ky[j + 1], m1 = km[j + 1];
  const double g = s.t1 - s.t0;
  const double ig = recip(g);
  const double ig6 = ig * (1.0 / 6.0);
  const double g26 = g * g * (1.0 / 6.0);
  s.a3 = m0 * ig6;
  s.b3 = m1 * ig6;
  s.p = fma(-m0, g26, y0) * ig;
  s.q = fma(-m1, g26, y1) * ig;
}

// Value at sample k; advances while t_{j+1} <= k (the last of the n knots
// lies beyond the signal, so the walk never passes it).
template <typename T>
__device__ __forceinline__ double seg_eval(Seg& s, const T* __restrict__ kt,
                                           const double* __restrict__ ky,
                                           const double* __restrict__ km, int n, double k) {
  while (s.t1 <= k && s.j + 2 < n) seg_load(s, kt, ky, km, s.j + 1);
  const double A = s.t1 - k, B = k - s.t0;
  const double A3 = A * A * A, B3 = B * B * B;
  return fma(s.a3, A3, fma(s.b3, B3, fma(s.p, A, s.q * B)));
}

}  // namespace dev
}  // namespace semd
