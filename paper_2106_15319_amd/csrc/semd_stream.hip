// Streaming (multi-workgroup) Serial-EMD kernels for gfx950, FP64.
//
// Signals too long for one workgroup's LDS are sifted in passes over global
// memory.  A batch's signals are cut into tiles of kTile samples; every tile
// kernel runs one workgroup per (signal, tile) pair of the whole batch, so a
// launch holds all the batch's parallelism.  One sift of every signal is
//   detect   (tiles)    extrema counts per tile, plus what the scan needs to
//                       resolve equal-valued runs that cross tile ends;
//   scan     (signals)  run-start carries and knot ranks across the tiles of
//                       a signal, knot totals, siftability, stop flags;
//   compact  (tiles)    knots (and mirrored end knots) written at their ranks;
//   solve    (blocks)   natural-spline second derivatives, blocks of knots
//                       staged in LDS, windowed Thomas sweeps per chunk;
//   eval     (tiles)    the tile's knots staged in LDS, both envelopes walked
//                       per thread, mean removed from h.
// Every signal carries its own phase (sift index, IMFs ended); the scan
// decides each step's action per signal, and the evaluation also performs
// IMF ends and final outputs, so signals in different phases share one
// step and finished ones are no-ops: a batch is K*S identical steps, and a
// serving engine admits new signals between steps.
#include <algorithm>

#include "semd_device.h"
#include "semd_stream.h"

namespace semd {
namespace {

using namespace dev;

constexpr int kTT = 256;              // threads per tile workgroup
constexpr int kTC = kTile / kTT;      // samples per thread
constexpr int kSB = kTT * kChunk;     // interior unknowns per solve block
constexpr int kTKnots = kTile / 2 + 8;  // knots of one kind a tile window can hold
constexpr int kNW = kTT / kWave;

__device__ __forceinline__ bool sifting(const SigStatus& st) {
  return st.action == kSift || st.action == kSiftLast;
}

// Block-wide reductions / scans over kTT threads (one barrier each, plus one
// on entry so the LDS scratch can be reused back to back).
__device__ __forceinline__ int block_max(int v, int* scratch) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v = max(v, __shfl_xor(v, d, kWave));
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  int m = scratch[0];
#pragma unroll
  for (int w = 1; w < kNW; ++w) m = max(m, scratch[w]);
  return m;
}

// Exclusive scans of one int64 per thread: sum (total returned) and max.
__device__ __forceinline__ int64_t block_excl_sum64(int64_t v, int64_t* scratch,
                                                    int64_t& total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int64_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t u = __shfl_up(inc, d, kWave);
    if (lane >= d) inc += u;
  }
  __syncthreads();
  if (lane == kWave - 1) scratch[wid] = inc;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kNW; ++w) {
    const int64_t a = scratch[w];
    before += (w < wid) ? a : 0;
    tot += a;
  }
  total = tot;
  return before + inc - v;
}

__device__ __forceinline__ int block_excl_max(int v, int* scratch, int& total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int u = __shfl_up(inc, d, kWave);
    if (lane >= d) inc = max(inc, u);
  }
  const int ex_in_wave = __shfl_up(inc, 1, kWave);
  __syncthreads();
  if (lane == kWave - 1) scratch[wid] = inc;
  __syncthreads();
  int before = -1, tot = -1;
#pragma unroll
  for (int w = 0; w < kNW; ++w) {
    const int a = scratch[w];
    if (w < wid) before = max(before, a);
    tot = max(tot, a);
  }
  total = tot;
  return lane > 0 ? max(before, ex_in_wave) : before;
}

// Stage samples a .. a+n-1 of h in LDS and return the halo neighbours.
__device__ __forceinline__ void stage_tile(const double* __restrict__ h, int a, int n, int L,
                                           double* tbuf, double& prev, double& next) {
  for (int i = threadIdx.x; i < n; i += kTT) tbuf[i] = h[a + i];
  prev = a > 0 ? h[a - 1] : 0.0;
  next = a + n < L ? h[a + n] : 0.0;
}

// ---------------------------------------------------------------------------
// Setup, load, detect, scan, compact
// ---------------------------------------------------------------------------

// Serialize (Sec. 3.2) and add the realization's noise (Sec. 2.2 Step 1):
// h = r = x for the tile; a non-finite sample marks the tile.
__global__ void __launch_bounds__(kTT) st_load_kernel(const StreamSig* __restrict__ sigs,
                                                      const int2* __restrict__ tiles) {
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  const int a = tv.y * kTile, b = min(a + kTile, S.L);
  const int64_t R = S.M + S.D;
  int bad = 0;
  for (int k = a + threadIdx.x; k < b; k += kTT) {
    const int64_t i = k / R, m = k - i * R;
    double v = serial_at(S.X, S.M, S.D, i, m);
    if (S.flags & 1) v = __dadd_rn(v, __dmul_rn(S.beta, noise_at(S.key, k)));
    bad |= !isfinite(v);
    S.h[k] = v;
    S.r[k] = v;
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    S.tinfo[tv.y].bad = bad ? 1 : 0;
    if (tv.y == 0) {
      SigStatus* st = S.st;
      st->active = 1;
      st->sift = 0;
      st->nimf = 0;
      st->bad = 0;
      st->action = kIdle;
      st->slot = 0;
      st->fin = 0;
      st->done = 0;
      st->n[0] = 0;
      st->n[1] = 0;
      st->n_sifts = 0;
      st->n_knots = 0;
    }
  }
}

// Extremum counts of a tile whose first run may have started in an earlier
// tile (kind kCont); that run's extremum, if any, is resolved by the scan.
__global__ void __launch_bounds__(kTT) st_detect_kernel(const StreamSig* __restrict__ sigs,
                                                        const int2* __restrict__ tiles) {
  __shared__ double tbuf[kTile];
  __shared__ double pub_first[kTT], pub_last[kTT];
  __shared__ int pub_key[kTT];
  __shared__ int scratch[kNW];
  __shared__ int64_t scratch64[kNW];
  __shared__ int cont_exit;
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  if (!S.st->active) return;
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  double prev, next;
  stage_tile(S.h, a, n, L, tbuf, prev, next);
  if (threadIdx.x == 0) cont_exit = 0;
  __syncthreads();
  const int first_key =
      a == 0 ? 0 : (prev != tbuf[0] ? a * 4 + step_kind(prev, tbuf[0]) : kCont);
  double h[kTC];
#pragma unroll
  for (int c = 0; c < kTC; ++c) {
    const int i = threadIdx.x * kTC + c;
    h[c] = i < n ? tbuf[i] : 0.0;
  }
  int carry, cmax, cmin, last;
  unsigned maxbits, minbits;
  detect_extrema<kTT, kTC>(h, a, n, L, threadIdx.x, first_key, next, pub_first, pub_last,
                           pub_key, carry, maxbits, minbits, cmax, cmin, &cont_exit, &last);
  int64_t tot;
  block_excl_sum64(((int64_t)cmax << 32) | (uint32_t)cmin, scratch64, tot);
  const int lastkey = block_max(last, scratch);
  if (threadIdx.x == 0) {
    TileInfo& t = S.tinfo[tv.y];
    t.cnt[0] = (int)(tot >> 32);
    t.cnt[1] = (int)(tot & 0xffffffff);
    t.lastkey = (lastkey & 3) == kCont ? -1 : lastkey;
    t.cont = first_key == kCont;
    t.cont_exit = cont_exit;
  }
}

// One workgroup per signal: carries and ranks across its tiles, knot totals,
// and the step's action (Sec. 2.1 Step 5 with a fixed sift count):
//   siftable candidate, sift < S-1  -> kSift
//   siftable candidate, sift = S-1  -> kSiftLast (the IMF ends after it)
//   not siftable, sift > 0          -> kEndImf   (the candidate is the IMF)
//   not siftable, sift = 0          -> kFinish   (the residue is final)
// An IMF end that reaches K IMFs also finishes the decomposition.
__global__ void __launch_bounds__(kTT) st_scan_kernel(const StreamSig* __restrict__ sigs) {
  __shared__ int64_t scratch64[kNW];
  __shared__ int scratch[kNW];
  const StreamSig& S = sigs[blockIdx.x];
  SigStatus* st = S.st;
  if (!st->active) {
    if (threadIdx.x == 0) st->action = kIdle;
    return;
  }
  const int nt = S.ntiles;
  // input with NaN/Inf: nothing is decomposed
  int bad = 0;
  for (int t = threadIdx.x; t < nt; t += kTT) bad |= S.tinfo[t].bad;
  bad = __syncthreads_or(bad);
  if (bad) {
    if (threadIdx.x == 0) {
      st->bad = 1;
      st->action = kFinish;
      st->fin = 1;
      st->active = 0;
    }
    return;
  }
  int carry_run = -1;
  int64_t off_run = 0;
  for (int t0 = 0; t0 < nt; t0 += kTT) {
    const int t = t0 + threadIdx.x;
    const bool valid = t < nt;
    TileInfo ti{};
    if (valid) ti = S.tinfo[t];
    int chunk_max;
    const int ex = block_excl_max(valid ? ti.lastkey : -1, scratch, chunk_max);
    const int carry_in = max(carry_run, ex);
    int dmax = 0, dmin = 0;
    if (valid && ti.cont) {
      const int entry = carry_in & 3;
      dmax = (ti.cont_exit == kFall && entry == kRise) ? 1 : 0;
      dmin = (ti.cont_exit == kRise && entry == kFall) ? 1 : 0;
    }
    const int tmax = valid ? ti.cnt[0] + dmax : 0, tmin = valid ? ti.cnt[1] + dmin : 0;
    int64_t chunk_tot;
    const int64_t ex_off =
        block_excl_sum64(((int64_t)tmax << 32) | (uint32_t)tmin, scratch64, chunk_tot);
    if (valid) {
      TileInfo& o = S.tinfo[t];
      o.carry = carry_in;
      o.tot[0] = tmax;
      o.tot[1] = tmin;
      const int64_t off = off_run + ex_off;
      o.off[0] = (int)(off >> 32);
      o.off[1] = (int)(off & 0xffffffff);
    }
    carry_run = max(carry_run, chunk_max);
    off_run += chunk_tot;
  }
  if (threadIdx.x == 0) {
    const int nmax = (int)(off_run >> 32), nmin = (int)(off_run & 0xffffffff);
    int action, fin = 0;
    if (nmax >= 1 && nmin >= 1 && nmax + nmin >= 3) {
      st->n[0] = nmax;
      st->n[1] = nmin;
      st->n_sifts += 1;
      st->n_knots += nmax + 2 * min(2, nmax) + nmin + 2 * min(2, nmin);
      action = st->sift + 1 >= S.S ? kSiftLast : kSift;
    } else {
      action = st->sift == 0 ? kFinish : kEndImf;
    }
    if (action == kSift) {
      st->sift += 1;
    } else if (action == kFinish) {
      fin = 1;
    } else {
      st->slot = st->nimf;
      st->nimf += 1;
      st->sift = 0;
      fin = st->nimf >= S.K;
    }
    st->action = action;
    st->fin = fin;
    if (fin) st->active = 0;
  }
}

// Knots of the tile at their ranks (Sec. 2.1 Step 1 -> Step 2).
__global__ void __launch_bounds__(kTT) st_compact_kernel(const StreamSig* __restrict__ sigs,
                                                         const int2* __restrict__ tiles) {
  __shared__ double tbuf[kTile];
  __shared__ double pub_first[kTT], pub_last[kTT];
  __shared__ int pub_key[kTT];
  __shared__ int64_t scratch64[kNW];
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  if (!sifting(*S.st)) return;
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  const TileInfo ti = S.tinfo[tv.y];
  double prev, next;
  stage_tile(S.h, a, n, L, tbuf, prev, next);
  __syncthreads();
  const int first_key =
      a == 0 ? 0 : (prev != tbuf[0] ? a * 4 + step_kind(prev, tbuf[0]) : ti.carry);
  double h[kTC];
#pragma unroll
  for (int c = 0; c < kTC; ++c) {
    const int i = threadIdx.x * kTC + c;
    h[c] = i < n ? tbuf[i] : 0.0;
  }
  int carry, cmax, cmin, last;
  unsigned maxbits, minbits;
  detect_extrema<kTT, kTC>(h, a, n, L, threadIdx.x, first_key, next, pub_first, pub_last,
                           pub_key, carry, maxbits, minbits, cmax, cmin, nullptr, &last);
  int64_t tot;
  const int64_t ex =
      block_excl_sum64(((int64_t)cmax << 32) | (uint32_t)cmin, scratch64, tot);
  const int nmax = S.st->n[0], nmin = S.st->n[1];
  const int base = a + threadIdx.x * kTC;
  const int nv = max(0, min(kTC, n - threadIdx.x * kTC));
  emit_knots<kTC>(h, maxbits, carry, base, nv, L, ti.off[0] + (int)(ex >> 32), nmax, S.kt[0],
                  S.ky[0], S.cap);
  emit_knots<kTC>(h, minbits, carry, base, nv, L, ti.off[1] + (int)(ex & 0xffffffff), nmin,
                  S.kt[1], S.ky[1], S.cap);
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------

// One block per (signal, envelope, kSB interior unknowns): the knots the
// block's chunks read (their rows plus kHalo+1 on each side) are staged in
// LDS, each thread solves one chunk and writes its second derivatives.
__global__ void __launch_bounds__(kTT) st_solve_kernel(const StreamSig* __restrict__ sigs,
                                                       const int4* __restrict__ blocks) {
  constexpr int kW = kSB + 2 * kHalo + 4;
  __shared__ int32_t lt[kW];
  __shared__ double ly[kW];
  const int4 bv = blocks[blockIdx.x];  // (signal, envelope, block)
  const StreamSig& S = sigs[bv.x];
  if (!sifting(*S.st)) return;
  const int env = bv.y;
  const int n = S.st->n[env];
  const int Pp = n < 2 ? n : 2;
  const int n2 = n + 2 * Pp;
  const int r0 = 1 + bv.z * kSB;
  if (n2 < 3 || r0 > n2 - 2) return;
  const int r1 = min(r0 + kSB, n2 - 1);  // rows r0 .. r1-1
  const int w0 = max(0, r0 - kHalo - 1), w1 = min(n2 - 1, r1 + kHalo);
  const int32_t* kt = S.kt[env];
  const double* ky = S.ky[env];
  for (int i = threadIdx.x; i <= w1 - w0; i += kTT) {
    lt[i] = kt[w0 + i];
    ly[i] = ky[w0 + i];
  }
  __syncthreads();
  const int ch = (r0 - 1) / kChunk + threadIdx.x;
  if (1 + ch * kChunk < r1) solve_chunk(lt, ly, w0, S.km[env], n2, ch);
  if (bv.z == 0 && threadIdx.x == 0) {
    S.km[env][0] = 0.0;
    S.km[env][n2 - 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Evaluate and update
// ---------------------------------------------------------------------------

// One step's work on the tile's samples:
//   kSift, kSiftLast  envelope means removed (Sec. 2.1 Steps 2-4): the knots
//                     whose segments cover the tile are staged in LDS and
//                     each thread walks them over its samples;
//   kSiftLast, kEndImf  IMF end: the candidate is stored in its output slot
//                     (deserialized, Sec. 3.3), r <- r - h, h <- r;
//   final             residue into slot K, unused IMF slots zero (Sec. 4.3),
//                     IMF count and statistics.
__global__ void __launch_bounds__(kTT) st_eval_kernel(const StreamSig* __restrict__ sigs,
                                                      const int2* __restrict__ tiles) {
  __shared__ double tbuf[kTile];
  __shared__ int32_t lt[2][kTKnots];
  __shared__ double ly[2][kTKnots], lm[2][kTKnots];
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  const SigStatus* st = S.st;
  const int action = st->action;
  if (action == kIdle) return;
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  for (int i = threadIdx.x; i < n; i += kTT) tbuf[i] = S.h[a + i];
  if (action == kSift || action == kSiftLast) {
    const TileInfo ti = S.tinfo[tv.y];
    int cnt[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int nk = st->n[e];
      const int Pp = nk < 2 ? nk : 2;
      const int n2 = nk + 2 * Pp;
      // the last knot emitted before the tile sits before it; the one after
      // the tile's first outside knot lies beyond the tile
      const int j0 = Pp + ti.off[e] - 1;
      const int j1 = min(n2 - 1, Pp + ti.off[e] + ti.tot[e] + 1);
      cnt[e] = min(j1 - j0 + 1, kTKnots);  // j1 - j0 <= kTile / 2 + 2 by the counts
      for (int i = threadIdx.x; i < cnt[e]; i += kTT) {
        lt[e][i] = S.kt[e][j0 + i];
        ly[e][i] = S.ky[e][j0 + i];
        lm[e][i] = S.km[e][j0 + i];
      }
    }
    __syncthreads();
    const int lb = threadIdx.x * kTC;
    const int nv = max(0, min(kTC, n - lb));
    if (nv > 0) {
      const double k0 = (double)(a + lb);
      Seg sg[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        // last window knot at or before the thread's first sample
        int lo = 0, hi = cnt[e] - 2;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if ((double)lt[e][mid] <= k0) lo = mid;
          else hi = mid - 1;
        }
        seg_load(sg[e], lt[e], ly[e], lm[e], lo);
      }
#pragma unroll 1
      for (int c = 0; c < nv; ++c) {
        const double kk = k0 + c;
        const double up = seg_eval(sg[0], lt[0], ly[0], lm[0], cnt[0], kk);
        const double lo = seg_eval(sg[1], lt[1], ly[1], lm[1], cnt[1], kk);
        const double mean = 0.5 * (up + lo);
        tbuf[lb + c] = tbuf[lb + c] - mean;
      }
    }
  }
  __syncthreads();
  const int64_t M = S.M, R = S.M + S.D, MN = S.M * S.N;
  if (action == kSiftLast || action == kEndImf) {
    double* slot = S.out + (int64_t)st->slot * MN;
    for (int i = threadIdx.x; i < n; i += kTT) {
      const int k = a + i;
      const double hk = tbuf[i];
      const double nr = S.r[k] - hk;
      S.r[k] = nr;
      tbuf[i] = nr;
      const int64_t ii = k / R, m = k - ii * R;
      if (m < M) slot[ii * M + m] = hk;
    }
  }
  if (st->fin) {
    const int K = S.K, bad = st->bad;
    const int nimf = bad ? 0 : st->nimf;
    for (int i = threadIdx.x; i < n; i += kTT) {
      const int k = a + i;
      const int64_t ii = k / R, m = k - ii * R;
      if (m < M) {
        const int64_t o = ii * M + m;
        for (int q = nimf; q < K; ++q) S.out[q * MN + o] = 0.0;
        S.out[(int64_t)K * MN + o] = bad ? 0.0 : tbuf[i];
      }
    }
    if (tv.y == 0 && threadIdx.x == 0) {
      if (S.n_imfs) *S.n_imfs = bad ? -5 : nimf;
      if (S.stats) {
        S.stats[0] = st->n_sifts;
        S.stats[1] = st->n_knots;
        S.stats[2] = st->n_sifts * (int64_t)S.L;
      }
      S.st->done = 1;
    }
  } else {
    for (int i = threadIdx.x; i < n; i += kTT) S.h[a + i] = tbuf[i];
  }
}

__global__ void st_gather_done_kernel(const StreamSig* __restrict__ sigs, int n,
                                      int32_t* __restrict__ done) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) done[i] = sigs[i].st->done;
}

inline dim3 per_signal(int n) { return dim3((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t st_load(const StreamSig* sigs, const int2* tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(st_load_kernel, dim3(ntiles), dim3(kTT), 0, s, sigs, tiles);
  return hipGetLastError();
}
hipError_t st_step(const StreamSig* sigs, int nsig, const int2* tiles, int ntiles,
                   const int4* blocks, int nblocks, hipStream_t st) {
  if (nsig <= 0) return hipSuccess;
  hipLaunchKernelGGL(st_detect_kernel, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  hipLaunchKernelGGL(st_scan_kernel, dim3(nsig), dim3(kTT), 0, st, sigs);
  hipLaunchKernelGGL(st_compact_kernel, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  hipLaunchKernelGGL(st_solve_kernel, dim3(nblocks), dim3(kTT), 0, st, sigs, blocks);
  hipLaunchKernelGGL(st_eval_kernel, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  return hipGetLastError();
}
hipError_t st_gather_done(const StreamSig* sigs, int nsig, int32_t* done, hipStream_t s) {
  if (nsig <= 0) return hipSuccess;
  hipLaunchKernelGGL(st_gather_done_kernel, per_signal(nsig), dim3(256), 0, s, sigs, nsig, done);
  return hipGetLastError();
}

int stream_solve_blocks(int cap) { return (cap + kSB - 1) / kSB; }

}  // namespace semd
