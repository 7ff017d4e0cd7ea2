// HIP kernels of the Serial-EMD hot path for gfx950 (MI355X), FP64 throughout.
//
// Resident path: one workgroup decomposes one serialized signal (or one EEMD
// realization) completely on chip.  The candidate h lives in registers in a
// blocked layout (thread t owns samples [t*C, t*C + C)); the knots of one
// envelope and their spline second derivatives live in LDS; the residue r is
// read and written once per IMF.  Per sift:
//   extrema (Sec. 2.1 Step 1)   neighbour exchange through LDS, plateau runs
//                                resolved by a walk over published run starts,
//                                per-thread counts, one block scan (wave
//                                shuffles + LDS wave totals) for compaction;
//   envelopes (Step 2)           knots + mirrored end knots written to LDS,
//                                natural-spline second derivatives by windowed
//                                Thomas sweeps (one thread per chunk of knots),
//                                evaluation by a per-thread walk over segments;
//   mean and update (Steps 3-4)  fused into the lower-envelope evaluation.
// Serialization (Sec. 3.2) and the EEMD noise (Sec. 2.2) are fused into the
// first load; deserialization (Sec. 3.3) into the IMF and residue stores.
#include <algorithm>

#include "semd_internal.h"

namespace semd {
namespace {

constexpr int kWave = 64;
constexpr int kChunk = 8;    // interior spline unknowns solved per thread
constexpr int kHalo = 32;    // knots swept on each side beyond a chunk
constexpr int kAggBytes = 256;
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

// ---------------------------------------------------------------------------
// Extrema (Sec. 2.1 Step 1) on the blocked register layout
// ---------------------------------------------------------------------------

// Each thread publishes its first and last sample and the key (4*index +
// step kind) of the last run start strictly inside its block; after one
// barrier every thread knows its neighbours and the start of the run its
// first sample belongs to.  A sample k <= L-2 where the run ends (h[k+1] !=
// h[k]) closes a maximum if the run was entered rising and is left falling
// (minimum: the reverse), at the floor-middle of the run.  Runs that start at
// sample 0 are entered with kind 0 and never yield an extremum; the run that
// ends at L-1 is never closed.
template <int NT, int C>
__device__ __forceinline__ void detect_extrema(const double (&h)[C], int base, int nv, int L,
                                               int tid, double* pub_first, double* pub_last,
                                               int* pub_key, int& carry, unsigned& maxbits,
                                               unsigned& minbits, int& cmax, int& cmin) {
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
  if (nv == C && base + C < L) next = pub_first[tid + 1];
  carry = 0;
  if (nv > 0 && base > 0) {
    const double prev = pub_last[tid - 1];
    if (prev != h[0]) {
      carry = base * 4 + step_kind(prev, h[0]);
    } else {
      // the run continues from an earlier block: walk back to its start
      int tau = tid - 1;
      for (;;) {
        const int kk = pub_key[tau];
        if (kk >= 0) { carry = kk; break; }
        if (tau == 0) { carry = 0; break; }
        const double pl = pub_last[tau - 1], pf = pub_first[tau];
        if (pl != pf) { carry = (tau * C) * 4 + step_kind(pl, pf); break; }
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
        }
      }
    }
  }
}

// Write this thread's knots of one kind (bits) at global ranks first.. among
// n, plus the mirrored end knots: the knot list is
//   [-k_P', ..., -k_1, k_1, ..., k_n, 2(L-1)-k_n, ..., 2(L-1)-k_{n-P'+1}],
// P' = min(2, n), mirrored knots carrying their source's value.
template <int C>
__device__ __forceinline__ void emit_knots(const double (&h)[C], unsigned bits, int carry,
                                           int base, int nv, int L, int first, int n,
                                           int16_t* kt, double* ky) {
  if (bits == 0u) return;
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
        kt[Pp + g] = (int16_t)mid;
        ky[Pp + g] = y;
        if (g == 0) { kt[Pp - 1] = (int16_t)(-mid); ky[Pp - 1] = y; }
        if (g == 1 && Pp == 2) { kt[0] = (int16_t)(-mid); ky[0] = y; }
        if (g == n - 1) { kt[Pp + n] = (int16_t)(hi - mid); ky[Pp + n] = y; }
        if (g == n - 2 && Pp == 2) { kt[Pp + n + 1] = (int16_t)(hi - mid); ky[Pp + n + 1] = y; }
        ++g;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Arithmetic helpers
// ---------------------------------------------------------------------------

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
__device__ __forceinline__ void solve_chunk(const int16_t* __restrict__ kt,
                                            const double* __restrict__ ky,
                                            double* __restrict__ km, int n, int ch) {
  const int s = 1 + ch * kChunk;
  const int e = min(s + kChunk - 1, n - 2);
  const int ws = max(1, s - kHalo);
  const int we = min(n - 2, e + kHalo);

  // forward sweep, positioned at row ws with row ws-1 standing in for the
  // coupling it drops (cp = dp = 0)
  double ftp = (double)kt[ws - 1], ft = (double)kt[ws];
  double fy = ky[ws];
  double fsp = (fy - ky[ws - 1]) * recip(ft - ftp);
  double cp = 0.0, dp = 0.0;
  // backward sweep, positioned at row we with row we+1 standing in likewise
  double btn = (double)kt[we + 1], bt = (double)kt[we];
  double by = ky[we];
  double bsn = (ky[we + 1] - by) * recip(btn - bt);
  double aa = 0.0, dd = 0.0;

  const int nf = s - ws;                    // forward halo rows ws .. s-1
  const int nb = (e < n - 2) ? we - e : 0;  // backward rows we .. e+1
  const int steps = max(nf, nb);
  for (int i = 0; i < steps; ++i) {
    if (i < nf) {
      const int j = ws + i;
      const double tn = (double)kt[j + 1], yn = ky[j + 1];
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
      const double tp = (double)kt[j - 1], yp = ky[j - 1];
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
      const double tn = (double)kt[j + 1], yn = ky[j + 1];
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
template <int NT>
__device__ void spline_second_derivs(const int16_t* __restrict__ kt,
                                     const double* __restrict__ ky, double* __restrict__ km,
                                     int n1, int o2, int n2, int tid) {
  const int c1 = n1 >= 3 ? (n1 - 2 + kChunk - 1) / kChunk : 0;
  const int c2 = n2 >= 3 ? (n2 - 2 + kChunk - 1) / kChunk : 0;
  for (int ch = tid; ch < c1 + c2; ch += NT) {
    const bool second = ch >= c1;
    const int o = second ? o2 : 0;
    solve_chunk(kt + o, ky + o, km + o, second ? n2 : n1, second ? ch - c1 : ch);
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

__device__ __forceinline__ void seg_load(Seg& s, const int16_t* __restrict__ kt,
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
__device__ __forceinline__ double seg_eval(Seg& s, const int16_t* __restrict__ kt,
                                           const double* __restrict__ ky,
                                           const double* __restrict__ km, int n, double k) {
  while (s.t1 <= k && s.j + 2 < n) seg_load(s, kt, ky, km, s.j + 1);
  const double A = s.t1 - k, B = k - s.t0;
  const double A3 = A * A * A, B3 = B * B * B;
  return fma(s.a3, A3, fma(s.b3, B3, fma(s.p, A, s.q * B)));
}

// ---------------------------------------------------------------------------
// Resident Serial-EMD kernel: one workgroup per work item
// ---------------------------------------------------------------------------

// LDS: 256 B of wave totals, then one area (area_bytes) used in turn as
//   - the staging buffer of the signal (L doubles) at load and IMF ends,
//   - the published block ends of the extremum detection (20 B per thread),
//   - the knot store: capk values, capk second derivatives, capk abscissae.
// A sift keeps both envelopes' knots in the store when they fit together
// (one solve, one fused evaluation and update); otherwise it builds them one
// after the other, parking the upper envelope in global memory.
template <int NT, int C>
__global__ void __launch_bounds__(NT) resident_emd_kernel(const WorkItem* __restrict__ items,
                                                          int K, int S, int area_bytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const WorkItem w = items[blockIdx.x];
  // the resident path holds at most kResidentMaxL samples: 32-bit indices
  const int L = w.L;
  const int M = (int)w.M, MN = (int)(w.M * w.N), R = (int)(w.M + w.D);
  const int D = w.D;

  int* wagg = reinterpret_cast<int*>(smem);
  unsigned char* area = smem + kAggBytes;
  const int capk = (area_bytes / (2 * (int)sizeof(double) + (int)sizeof(int16_t))) & ~7;
  double* stage = reinterpret_cast<double*>(area);
  double* ky = reinterpret_cast<double*>(area);
  double* km = ky + capk;
  int16_t* kt = reinterpret_cast<int16_t*>(km + capk);
  double* pub_first = reinterpret_cast<double*>(area);
  double* pub_last = pub_first + NT;
  int* pub_key = reinterpret_cast<int*>(pub_last + NT);

  const int base = tid * C;
  const int nv = max(0, min(C, L - base));

  // Load: serialize (Sec. 3.2), add the realization's noise (Sec. 2.2 Step 1)
  int bad = 0;
  for (int k = tid; k < L; k += NT) {
    const int i = k / R, m = k - i * R;
    double v = serial_at(w.X, M, D, i, m);
    if (w.flags & 1) v = __dadd_rn(v, __dmul_rn(w.beta, noise_at(w.key, k)));
    bad |= !isfinite(v);
    stage[k] = v;
    w.r[k] = v;
  }
  if (__syncthreads_or(bad)) {
    for (int64_t o = tid; o < (int64_t)(K + 1) * MN; o += NT) w.out[o] = 0.0;
    if (tid == 0 && w.n_imfs) *w.n_imfs = -5;
    return;
  }
  double h[C];
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = (c < nv) ? stage[base + c] : 0.0;

  int nimf = 0;
  int64_t n_sifts = 0, n_knots = 0;
  while (nimf < K) {
    bool stop = false;
    for (int s = 0; s < S; ++s) {
      __syncthreads();  // previous readers of the LDS area are done
      int carry, cmax, cmin;
      unsigned maxbits, minbits;
      detect_extrema<NT, C>(h, base, nv, L, tid, pub_first, pub_last, pub_key, carry, maxbits,
                            minbits, cmax, cmin);
      int tot;
      const int excl = block_excl_sum<NW>((cmax << 16) | cmin, wagg, lane, wid, tot);
      const int nmax = tot >> 16, nmin = tot & 0xffff;
      if (!(nmax >= 1 && nmin >= 1 && nmax + nmin >= 3)) {
        stop = (s == 0);  // the residue itself is not siftable: decomposition ends
        break;
      }
      const int emax = excl >> 16, emin = excl & 0xffff;
      const int pmax = nmax < 2 ? nmax : 2, pmin = nmin < 2 ? nmin : 2;
      const int nkmax = nmax + 2 * pmax, nkmin = nmin + 2 * pmin;
      ++n_sifts;
      n_knots += nkmax + nkmin;
      if (nkmax + nkmin <= capk) {
        // both envelopes at once
        emit_knots<C>(h, maxbits, carry, base, nv, L, emax, nmax, kt, ky);
        emit_knots<C>(h, minbits, carry, base, nv, L, emin, nmin, kt + nkmax, ky + nkmax);
        __syncthreads();
        spline_second_derivs<NT>(kt, ky, km, nkmax, nkmax, nkmin, tid);
        __syncthreads();
        if (nv > 0) {
          Seg su, sl;
          seg_load(su, kt, ky, km, pmax + emax - 1);
          seg_load(sl, kt + nkmax, ky + nkmax, km + nkmax, pmin + emin - 1);
#pragma unroll 1
          for (int c = 0; c < C; ++c) {
            if (c < nv) {
              const double kk = (double)(base + c);
              const double up = seg_eval(su, kt, ky, km, nkmax, kk);
              const double lo = seg_eval(sl, kt + nkmax, ky + nkmax, km + nkmax, nkmin, kk);
              const double mean = 0.5 * (up + lo);
              h[c] = h[c] - mean;
            }
          }
        }
      } else {
        // one envelope at a time
        emit_knots<C>(h, maxbits, carry, base, nv, L, emax, nmax, kt, ky);
        __syncthreads();
        spline_second_derivs<NT>(kt, ky, km, nkmax, 0, 0, tid);
        __syncthreads();
        if (nv > 0) {
          Seg su;
          seg_load(su, kt, ky, km, pmax + emax - 1);
#pragma unroll 1
          for (int c = 0; c < C; ++c)
            if (c < nv) w.u[base + c] = seg_eval(su, kt, ky, km, nkmax, (double)(base + c));
        }
        __syncthreads();
        emit_knots<C>(h, minbits, carry, base, nv, L, emin, nmin, kt, ky);
        __syncthreads();
        spline_second_derivs<NT>(kt, ky, km, nkmin, 0, 0, tid);
        __syncthreads();
        if (nv > 0) {
          Seg sl;
          seg_load(sl, kt, ky, km, pmin + emin - 1);
#pragma unroll 1
          for (int c = 0; c < C; ++c) {
            if (c < nv) {
              const double lo = seg_eval(sl, kt, ky, km, nkmin, (double)(base + c));
              const double mean = 0.5 * (w.u[base + c] + lo);
              h[c] = h[c] - mean;
            }
          }
        }
      }
    }
    if (stop) break;
    // IMF nimf = h (deserialized store, Sec. 3.3); residue r <- r - h
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (c < nv) stage[base + c] = h[c];
    __syncthreads();
    double* slot = w.out + (int64_t)nimf * MN;
    for (int k = tid; k < L; k += NT) {
      const double hk = stage[k];
      const double nr = w.r[k] - hk;
      w.r[k] = nr;
      stage[k] = nr;
      const int i = k / R, m = k - i * R;
      if (m < M) slot[i * M + m] = hk;
    }
    ++nimf;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) h[c] = (c < nv) ? stage[base + c] : 0.0;
  }
  // residue into slot K, unused IMF slots zero (Sec. 4.3 zero fill)
  double* rslot = w.out + (int64_t)K * MN;
  for (int k = tid; k < L; k += NT) {
    const int i = k / R, m = k - i * R;
    if (m < M) rslot[i * M + m] = w.r[k];
  }
  for (int64_t o = (int64_t)nimf * MN + tid; o < (int64_t)K * MN; o += NT) w.out[o] = 0.0;
  if (tid == 0 && w.n_imfs) *w.n_imfs = nimf;
  if (tid == 0 && w.stats) {
    w.stats[0] = n_sifts;
    w.stats[1] = n_knots;
    w.stats[2] = n_sifts * (int64_t)L;
  }
}

template <int NT, int C>
__global__ void __launch_bounds__(NT) extrema_kernel(const double* __restrict__ hin, int L,
                                                     int32_t* __restrict__ imax,
                                                     int32_t* __restrict__ imin,
                                                     int32_t* __restrict__ counts) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  int* wagg = reinterpret_cast<int*>(smem);
  double* pub_first = reinterpret_cast<double*>(smem + kAggBytes);
  double* pub_last = pub_first + NT;
  int* pub_key = reinterpret_cast<int*>(pub_last + NT);
  const int base = tid * C;
  const int nv = max(0, min(C, L - base));
  double h[C];
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = (c < nv) ? hin[base + c] : 0.0;
  int carry, cmax, cmin;
  unsigned maxbits, minbits;
  detect_extrema<NT, C>(h, base, nv, L, tid, pub_first, pub_last, pub_key, carry, maxbits,
                        minbits, cmax, cmin);
  int tot;
  const int excl = block_excl_sum<NW>((cmax << 16) | cmin, wagg, lane, wid, tot);
  int gmax = excl >> 16, gmin = excl & 0xffff;
  int start = carry >> 2;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if (c < nv) {
      const int k = base + c;
      if (c > 0 && h[c - 1] != h[c]) start = k;
      const int mid = (start + k) >> 1;
      if ((maxbits >> c) & 1u) imax[gmax++] = mid;
      if ((minbits >> c) & 1u) imin[gmin++] = mid;
    }
  }
  if (tid == 0) {
    counts[0] = tot >> 16;
    counts[1] = tot & 0xffff;
  }
}

// ---------------------------------------------------------------------------
// Streaming helper kernels
// ---------------------------------------------------------------------------

__global__ void serialize_kernel(const double* __restrict__ X, int64_t M, int64_t N, int D,
                                 double* __restrict__ x) {
  const int64_t R = M + D, L = M * N + (int64_t)D * N - D;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k / R, m = k - i * R;
    x[k] = serial_at(X, M, D, i, m);
  }
}

__global__ void deserialize_kernel(const double* __restrict__ y, int64_t M, int64_t N, int D,
                                   double* __restrict__ out) {
  const int64_t R = M + D;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < M * N;
       o += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = o / M, m = o - i * M;
    out[o] = y[i * R + m];
  }
}

__global__ void noise_kernel(uint64_t key, int64_t L, double* __restrict__ w) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L;
       k += (int64_t)gridDim.x * blockDim.x)
    w[k] = noise_at(key, k);
}

__global__ void ensemble_mean_kernel(const double* __restrict__ src, int NR, int64_t count,
                                     double* __restrict__ dst) {
  const double den = (double)NR;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < NR; ++m) acc = acc + src[(int64_t)m * count + i];
    dst[i] = acc / den;
  }
}

__global__ void max_count_kernel(const int32_t* __restrict__ n_src, int NR,
                                 int32_t* __restrict__ n_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int32_t best = 0, err = 0;
    for (int m = 0; m < NR; ++m) {
      const int32_t v = n_src[m];
      if (v < 0) err = v;
      else if (v > best) best = v;
    }
    *n_out = err < 0 ? err : best;
  }
}

inline int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

template <int NT, int C>
hipError_t launch_resident_cls(const WorkItem* d_items, int n, int maxL, int K, int S,
                               hipStream_t stream) {
  auto kern = resident_emd_kernel<NT, C>;
  // LDS per workgroup is 160 KiB, shared with the kernel's static LDS
  static const int static_lds = [&] {
    hipFuncAttributes a{};
    return hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kern)) == hipSuccess
               ? (int)a.sharedSizeBytes
               : 1024;
  }();
  const size_t limit = 160 * 1024 - (size_t)static_lds;
  const size_t area = resident_area_bytes(maxL, NT, limit - kAggBytes);
  const size_t lds = kAggBytes + area;
  if (lds > limit) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(NT), lds, stream, d_items, K, S, (int)area);
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Threads and samples per thread for signals up to maxL samples.
ResidentClass resident_class(int maxL) {
  if (maxL <= 256 * 4) return {256, 4};
  if (maxL <= 256 * 8) return {256, 8};
  if (maxL <= 256 * 12) return {256, 12};
  if (maxL <= 256 * 16) return {256, 16};
  if (maxL <= 512 * 12) return {512, 12};
  if (maxL <= 512 * 16) return {512, 16};
  if (maxL <= 1024 * 12) return {1024, 12};
  return {1024, 16};
}

size_t resident_area_bytes(int maxL, int nt, size_t max_area) {
  const size_t per_knot = 2 * sizeof(double) + sizeof(int16_t);
  const size_t stage = (size_t)maxL * sizeof(double);
  const size_t pub = (size_t)nt * (2 * sizeof(double) + sizeof(int));
  // one envelope at a time must always fit (at most (L-1)/2 + 4 knots each)
  const size_t single = per_knot * ((size_t)knot_cap(maxL) + 8);
  // both envelopes together (at most L + 6 knots) when the budget allows:
  // 2 workgroups per CU below 1024 threads, one above
  const size_t dual = per_knot * ((size_t)maxL + 16);
  const size_t budget = std::min(max_area, nt >= 1024 ? max_area : max_area / 2 - 512);
  size_t area = std::min(dual, budget);
  area = std::max(area, std::max(stage, std::max(pub, single)));
  return align16(area) <= max_area ? align16(area) : max_area & ~size_t(15);
}

hipError_t launch_resident(const WorkItem* d_items, int n, int maxL, int K, int S,
                           hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const ResidentClass c = resident_class(maxL);
  switch (c.nt * 100 + c.c) {
    case 25604: return launch_resident_cls<256, 4>(d_items, n, maxL, K, S, stream);
    case 25608: return launch_resident_cls<256, 8>(d_items, n, maxL, K, S, stream);
    case 25612: return launch_resident_cls<256, 12>(d_items, n, maxL, K, S, stream);
    case 25616: return launch_resident_cls<256, 16>(d_items, n, maxL, K, S, stream);
    case 51212: return launch_resident_cls<512, 12>(d_items, n, maxL, K, S, stream);
    case 51216: return launch_resident_cls<512, 16>(d_items, n, maxL, K, S, stream);
    case 102412: return launch_resident_cls<1024, 12>(d_items, n, maxL, K, S, stream);
    default: return launch_resident_cls<1024, 16>(d_items, n, maxL, K, S, stream);
  }
}

hipError_t launch_extrema(const double* h, int L, int32_t* imax, int32_t* imin,
                          int32_t* counts, hipStream_t stream) {
  constexpr int NT = 1024, C = 16;
  const size_t lds = kAggBytes + align16((size_t)NT * (2 * sizeof(double) + sizeof(int)));
  hipLaunchKernelGGL((extrema_kernel<NT, C>), dim3(1), dim3(NT), lds, stream, h, L, imax, imin,
                     counts);
  return hipGetLastError();
}

hipError_t launch_serialize(const double* X, int64_t M, int64_t N, int D, double* x,
                            hipStream_t stream) {
  const int64_t L = M * N + (int64_t)D * N - D;
  hipLaunchKernelGGL(serialize_kernel, dim3(grid_for(L, 256)), dim3(256), 0, stream, X, M, N,
                     D, x);
  return hipGetLastError();
}

hipError_t launch_deserialize(const double* y, int64_t M, int64_t N, int D, double* out,
                              hipStream_t stream) {
  hipLaunchKernelGGL(deserialize_kernel, dim3(grid_for(M * N, 256)), dim3(256), 0, stream, y,
                     M, N, D, out);
  return hipGetLastError();
}

hipError_t launch_noise(uint64_t key, int64_t L, double* w, hipStream_t stream) {
  hipLaunchKernelGGL(noise_kernel, dim3(grid_for(L, 256)), dim3(256), 0, stream, key, L, w);
  return hipGetLastError();
}

hipError_t launch_ensemble_mean(const double* src, int NR, int64_t count, double* dst,
                                hipStream_t stream) {
  hipLaunchKernelGGL(ensemble_mean_kernel, dim3(grid_for(count, 256)), dim3(256), 0, stream,
                     src, NR, count, dst);
  return hipGetLastError();
}

hipError_t launch_max_count(const int32_t* n_src, int NR, int32_t* n_out, hipStream_t stream) {
  hipLaunchKernelGGL(max_count_kernel, dim3(1), dim3(64), 0, stream, n_src, NR, n_out);
  return hipGetLastError();
}

}  // namespace semd
