// Streaming (multi-workgroup) Serial-EMD kernels for gfx950, FP64.
//
// Signals too long for one workgroup's LDS are sifted in passes over global
// memory.  A batch's signals are cut into tiles of kTile samples; every tile
// kernel runs one workgroup per (signal, tile) pair of the whole batch, so a
// launch holds all the batch's parallelism.  A step starts with the extrema
// of every tile's candidate detected (extrema counts and lists per tile,
// plus what the scan needs to resolve equal-valued runs that cross tile
// ends), by the load or the previous step's evaluation.  One sift of every
// signal is
//   scan     (signals)  run-start carries and knot ranks across the tiles of
//                       a signal, knot totals, siftability, stop flags;
//   compact  (tiles)    knots (and mirrored end knots) written at their ranks;
//   solve    (blocks)   natural-spline second derivatives and segment
//                       records, each block's window of knots staged in LDS
//                       and solved exactly by block-wide scans;
//   eval     (tiles)    both envelopes walked per thread over the segment
//                       records, mean removed from h, IMF ends, and the next
//                       candidate's extrema detected while it is on chip.
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

constexpr int kTT = kTileThreads;     // threads per tile workgroup
constexpr int kTC = kTile / kTT;      // samples per thread
constexpr int kSB = 1536;             // interior rows per solve block
// An envelope's solve blocks are sized for its largest possible knot count
// (about L/2), and in most sifts most of them are empty.  A launch over many
// blocks folds them: each workgroup takes every G-th block of its envelope,
// so an empty block costs a loop test instead of a workgroup.  The fold
// (kSolveTarget unfolded blocks per workgroup slot, at most kSolveFoldMax)
// leaves a launch over few signals unfolded, so it keeps its parallelism.
constexpr int kSolveTarget = 4096;
constexpr int kSolveFoldMax = 32;
__host__ __device__ constexpr int solve_blocks(int cap) { return (cap + kSB - 1) / kSB; }
// Solve blocks per workgroup of a folded launch over `units` blocks.
inline int launch_fold(int64_t units, int target = kSolveTarget) {
  return (int)std::min<int64_t>(kSolveFoldMax, std::max<int64_t>(1, units / target));
}
constexpr int kNW = kTT / kWave;
constexpr int kCompactWaves = 4;  // tiles per compaction workgroup, one wave each
constexpr int kCompactBatch = 4;  // list entries per lane and list loaded per round
constexpr int kCompactThreads = kWave * kCompactWaves;

template <class Status>
__device__ __forceinline__ bool sifting(const Status& st) {
  return st.action == kSift || st.action == kSiftLast;
}

// Inclusive scans within a wave by DPP moves (Kogge-Stone within each row of
// 16 lanes, then the row totals broadcast down the wave): maximum, sum.
constexpr int kIntMin = -2147483647 - 1;
__device__ __forceinline__ int wave_incl_max(int v) {
  v = max(v, dpp_int<kDppRowShr + 1, 0xf, kIntMin>(v));
  v = max(v, dpp_int<kDppRowShr + 2, 0xf, kIntMin>(v));
  v = max(v, dpp_int<kDppRowShr + 4, 0xf, kIntMin>(v));
  v = max(v, dpp_int<kDppRowShr + 8, 0xf, kIntMin>(v));
  v = max(v, dpp_int<kDppRowBcast15, 0xa, kIntMin>(v));
  v = max(v, dpp_int<kDppRowBcast31, 0xc, kIntMin>(v));
  return v;
}
__device__ __forceinline__ int64_t wave_incl_sum64(int64_t v) {
  v += dpp_i64<kDppRowShr + 1, 0xf>(v);
  v += dpp_i64<kDppRowShr + 2, 0xf>(v);
  v += dpp_i64<kDppRowShr + 4, 0xf>(v);
  v += dpp_i64<kDppRowShr + 8, 0xf>(v);
  v += dpp_i64<kDppRowBcast15, 0xa>(v);
  v += dpp_i64<kDppRowBcast31, 0xc>(v);
  return v;
}

// Block-wide reductions / scans over kTT threads (one barrier each, plus one
// on entry so the LDS scratch can be reused back to back).
__device__ __forceinline__ int block_max(int v, int* scratch) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  v = wave_incl_max(v);
  __syncthreads();
  if (lane == kWave - 1) scratch[wid] = v;
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
  const int64_t inc = wave_incl_sum64(v);
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
  const int inc = wave_incl_max(v);
  const int ex_in_wave = dpp_int<kDppWaveShr1, 0xf, kIntMin>(inc);  // (lane 0: unused)
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

// Position of tile sample i in the LDS tile buffer: within each block of
// kTC = 8 samples (one thread's), the sample index is XORed with bits 2..4
// of the block index, so that the threads' blocked accesses (stride 8
// doubles) fall on distinct banks for 32 lanes, while consecutive samples
// stay within their block.
static_assert(kTC == 8, "tile buffer swizzle assumes 8 samples per thread");
__device__ __forceinline__ int tsw(int i) { return i ^ ((i >> 5) & 7); }

// Two consecutive samples (or knot values), moved by one 16-byte access,
// and two consecutive knot positions.
struct alignas(16) SamplePair {
  double x, y;
};
struct alignas(8) RankPair {
  int32_t x, y;
};

// Samples 0..n-1 of the tile buffer to dst (a tile's first sample: 16-byte
// aligned), in sample pairs.
__device__ __forceinline__ void store_tile(global_ptr<double> dst, int n, const double* tbuf) {
  const global_ptr<SamplePair> d2 = (global_ptr<SamplePair>)dst;
  for (int j = threadIdx.x; j < n / 2; j += kTileThreads) {
    const int s0 = tsw(2 * j);
    auto& d = d2[j];  // (one 16-byte store)
    d.x = tbuf[s0];
    d.y = tbuf[s0 ^ 1];
  }
  if ((n & 1) && threadIdx.x == 0) dst[n - 1] = tbuf[tsw(n - 1)];
}

// ---------------------------------------------------------------------------
// Extrema of a tile (Sec. 2.1 Step 1) from per-thread step masks
// ---------------------------------------------------------------------------

// What the detection of one thread's samples yields.
struct TileDet {
  unsigned maxbits, minbits;  // the thread's samples closing a maximum / minimum run
  unsigned NE;                // bit b: sample b differs from sample b-1 (run starts)
  int carry;                  // key of the run holding the thread's first sample
  int last;                   // key of the run holding its last sample (-1: none)
};

// A tile holds samples a .. a+n-1 of a signal of length L; thread t owns the
// C samples from a + t*C in h[].  first_key is the key (4*start + kind) of
// the run holding sample a: 0 at the signal start (kind 0, never an
// extremum), a*4 + kind when sample a differs from sample a-1, else the key
// of a run that started before the tile, or kCont when that key is unknown
// (its extremum, if any, is then left to the scan: the direction the run is
// left in is written to *cont_exit, the sample it ends at to *cont_pos and
// its value to *cont_y).  next is sample a+n when a+n < L.  The tile buffer
// tb holds the same samples (swizzled positions), from which the
// neighbouring threads' first and last samples are read.
// Bit b of the rise (fall) mask marks sample b above (below) sample b-1, bit
// C the step to the next thread's first sample; a sample closes a run when
// its next step is not flat, and the run is a maximum when entered rising
// and left falling (minimum: the reverse).  Contains one barrier.
template <int C>
__device__ __forceinline__ void tile_detect(const double (&h)[C], int a, int n, int L, int tid,
                                            int first_key, double next, const double* tb,
                                            int* pub_key, int* cont_exit, int* cont_pos,
                                            double* cont_y, TileDet& d) {
  const int lb = tid * C, base = a + lb;
  // first and last sample of thread t's block (t holding at least one)
  auto first_of = [&](int t) { return tb[tsw(t * C)]; };
  auto last_of = [&](int t) { return tb[tsw(min(t * C + C, n) - 1)]; };
  const int nv = max(0, min(C, n - lb));
  unsigned R = 0u, F = 0u;
#pragma unroll
  for (int b = 1; b < C; ++b) {
    if (b < nv) {
      R |= (h[b] > h[b - 1] ? 1u : 0u) << b;
      F |= (h[b] < h[b - 1] ? 1u : 0u) << b;
    }
  }
  if (nv > 0) {
    const unsigned inner = R | F;
    int key = -1;
    if (inner) {
      const int b = 31 - __clz(inner);
      key = (base + b) * 4 + (((R >> b) & 1u) ? kRise : kFall);
    }
    pub_key[tid] = key;
  }
  __syncthreads();
  d.maxbits = 0u;
  d.minbits = 0u;
  d.NE = 0u;
  d.carry = first_key;
  d.last = -1;
  if (nv <= 0) return;
  int carry = first_key;
  if (tid > 0) {
    const double prev = last_of(tid - 1);
    R |= h[0] > prev ? 1u : 0u;
    F |= h[0] < prev ? 1u : 0u;
    if (prev != h[0]) {
      carry = base * 4 + step_kind(prev, h[0]);
    } else {
      // the run continues from an earlier thread: walk back to its start
      int tau = tid - 1;
      for (;;) {
        const int kk = pub_key[tau];
        if (kk >= 0) { carry = kk; break; }
        if (tau == 0) { carry = first_key; break; }
        const double pl = last_of(tau - 1), pf = first_of(tau);
        if (pl != pf) { carry = (a + tau * C) * 4 + step_kind(pl, pf); break; }
        --tau;
      }
    }
  } else if (a > 0 && (first_key >> 2) == a) {
    // sample a starts a run: the step into it
    R |= (first_key & 3) == kRise ? 1u : 0u;
    F |= (first_key & 3) == kFall ? 1u : 0u;
  }
  if (nv == C && base + C < L) {
    const double nx = (lb + C < n) ? first_of(tid + 1) : next;
    R |= (nx > h[C - 1] ? 1u : 0u) << C;
    F |= (nx < h[C - 1] ? 1u : 0u) << C;
  }
  const unsigned NE = R | F;
  const unsigned valid = (1u << nv) - 1u;
  unsigned maxbits = R & (F >> 1) & valid;
  unsigned minbits = F & (R >> 1) & valid;
  unsigned pe = (NE >> 1) & ~NE & valid;
  while (pe) {
    const int c = __ffs(pe) - 1;
    pe &= pe - 1u;
    const unsigned below = NE & ((1u << c) - 1u);
    int kind;
    if (below) {
      const int b = 31 - __clz(below);
      kind = ((R >> b) & 1u) ? kRise : kFall;
    } else {
      kind = carry & 3;
    }
    if (kind == kRise && ((F >> (c + 1)) & 1u)) maxbits |= 1u << c;
    else if (kind == kFall && ((R >> (c + 1)) & 1u)) minbits |= 1u << c;
    else if (kind == kCont && cont_exit) {
      *cont_exit = ((F >> (c + 1)) & 1u) ? kFall : kRise;
      *cont_pos = base + c;
      *cont_y = h[c];
    }
  }
  const unsigned top = NE & valid;
  if (top) {
    const int b = 31 - __clz(top);
    d.last = (base + b) * 4 + (((R >> b) & 1u) ? kRise : kFall);
  } else {
    d.last = carry;
  }
  d.maxbits = maxbits;
  d.minbits = minbits;
  d.NE = NE;
  d.carry = carry;
}

// Floor-middle of the equal-valued run that sample c of a thread closes
// (NE and carry as in TileDet; base is the thread's first sample).
__device__ __forceinline__ int run_mid(unsigned NE, int carry, int base, int c) {
  const unsigned below = NE & ((2u << c) - 1u);
  const int start = below ? base + (31 - __clz(below)) : (carry >> 2);
  return (start + base + c) >> 1;
}

// What detection leaves for the scan, compaction and evaluation: each
// thread's knots at tile-local ranks (positions and values), the knots each
// thread's predecessors in the tile hold, the tile's counts and run keys, and
// the continued run's end (its extremum is decided by the scan).  The knot
// lists are assembled in `stage` (LDS of kTile doubles, free on entry), one
// kind at a time, and written out as contiguous runs: written straight from
// the threads, each store instruction would touch many partly written
// cache lines.
__device__ __forceinline__ void record_tile(const TileDet& d, const double (&h)[kTC], int a,
                                            int first_key, int cont_exit, int cont_pos,
                                            double cont_y, const StreamSig& S, int tile,
                                            int64_t* scratch64, int* scratch, double* stage) {
  int64_t tot;
  const int64_t ex = block_excl_sum64(
      ((int64_t)__popc(d.maxbits) << 32) | (uint32_t)__popc(d.minbits), scratch64, tot);
  const int g0[2] = {(int)(ex >> 32), (int)(ex & 0xffffffff)};
  const int cnt[2] = {(int)(tot >> 32), (int)(tot & 0xffffffff)};
  // (tile-local ranks are below 2^16: maxima in the low half, minima high)
  gmem(S.trank)[(int64_t)tile * kTT + threadIdx.x] = (int32_t)((uint32_t)g0[0] |
                                                               ((uint32_t)g0[1] << 16));
  const int base = a + threadIdx.x * kTC;
  const int64_t lo = (int64_t)tile * kTileKnots;
  static_assert(kTileKnots < (1 << 16), "tile-local ranks fit 16 bits");
  static_assert(kTileKnots * (sizeof(double) + sizeof(int32_t)) <= kTile * sizeof(double),
                "one kind's knot list fits the staging area");
  double* sval = stage;
  int32_t* spos = reinterpret_cast<int32_t*>(stage + kTileKnots);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const unsigned bits = e ? d.minbits : d.maxbits;
    int g = g0[e];
    __syncthreads();  // the staging area is free (tile buffer or previous kind)
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      if ((bits >> c) & 1u) {
        spos[g] = run_mid(d.NE, d.carry, base, c);
        sval[g] = h[c];
        ++g;
      }
    }
    __syncthreads();
    const global_ptr<int32_t> lp = gmem(S.lpos[e]) + lo;
    const global_ptr<double> lv = gmem(S.lval[e]) + lo;
    for (int i = threadIdx.x; i < cnt[e]; i += kTT) {
      lp[i] = spos[i];
      lv[i] = sval[i];
    }
  }
  const int lastkey = block_max(d.last, scratch);
  if (threadIdx.x == 0) {
    auto& t = gmem(S.tinfo)[tile];
    t.cnt[0] = (int)(tot >> 32);
    t.cnt[1] = (int)(tot & 0xffffffff);
    t.lastkey = (lastkey & 3) == kCont ? -1 : lastkey;
    t.cont = first_key == kCont;
    t.cont_exit = cont_exit;
    t.cont_pos = cont_exit ? cont_pos : -1;
    t.cont_y = cont_y;
  }
}

// ---------------------------------------------------------------------------
// Setup, load, scan, compact
// ---------------------------------------------------------------------------

// Extremum detection of a tile staged in tbuf (samples a .. a+n-1), its
// neighbours' samples being prev and next (0 where the signal ends).
__device__ __forceinline__ void detect_staged(const StreamSig& S, int tile, int a, int n,
                                              double prev, double next, double* tbuf,
                                              int* pub_key, int* scratch, int64_t* scratch64,
                                              int& cont_exit, int& cont_pos, double& cont_y) {
  const int L = S.L;
  if (threadIdx.x == 0) cont_exit = 0;
  __syncthreads();
  const int first_key =
      a == 0 ? 0 : (prev != tbuf[tsw(0)] ? a * 4 + step_kind(prev, tbuf[tsw(0)]) : kCont);
  double h[kTC];
#pragma unroll
  for (int c = 0; c < kTC; ++c) {
    const int i = threadIdx.x * kTC + c;
    h[c] = i < n ? tbuf[tsw(i)] : 0.0;
  }
  TileDet d;
  tile_detect<kTC>(h, a, n, L, threadIdx.x, first_key, next, tbuf, pub_key,
                   &cont_exit, &cont_pos, &cont_y, d);
  __syncthreads();
  record_tile(d, h, a, first_key, cont_exit, cont_pos, cont_y, S, tile, scratch64, scratch,
              tbuf);
}

// Serialize (Sec. 3.2) and add the realization's noise (Sec. 2.2 Step 1):
// r = x for the tile (the first step reads its candidate h = r there); a
// non-finite sample marks the tile.  The tile's
// extrema are detected while it is on chip (the neighbours' samples are
// computed alongside).
__global__ void __launch_bounds__(kTT) st_load_kernel(const StreamSig* __restrict__ sigs,
                                                      const int2* __restrict__ tiles) {
  __shared__ double tbuf[kTile];
  __shared__ int pub_key[kTT];
  __shared__ int scratch[kNW];
  __shared__ int64_t scratch64[kNW];
  __shared__ int cont_exit, cont_pos;
  __shared__ double cont_y;
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  const int64_t R = S.M + S.D;
  auto sample = [&](int k) {
    const int64_t i = k / R, m = k - i * R;
    double v = (S.flags & kNoSignal) ? 0.0 : serial_at(S.X, S.M, S.D, i, m);
    if (S.flags & (kAddNoise | kAddBuffer)) {
      const double b = (S.flags & kScaleOnDevice) ? *S.scale : S.beta;
      const double e = (S.flags & kAddNoise) ? noise_at(S.key, k) : S.addend[k];
      v = __dadd_rn(v, __dmul_rn(b, e));
    }
    return v;
  };
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += kTT) {
    const double v = sample(a + i);
    bad |= !isfinite(v);
    S.r[a + i] = v;
    tbuf[tsw(i)] = v;
  }
  const double prev = a > 0 ? sample(a - 1) : 0.0;
  const double next = a + n < L ? sample(a + n) : 0.0;
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
      st->in_r = 0;
    }
  }
  detect_staged(S, tv.y, a, n, prev, next, tbuf, pub_key, scratch, scratch64, cont_exit,
                cont_pos, cont_y);
}

// Ends the current IMF (its candidate is stored by the evaluation); reaching
// K IMFs finishes the decomposition.
__device__ __forceinline__ void end_imf(SigStatus* st, int K) {
  st->slot = st->nimf;
  st->nimf += 1;
  st->sift = 0;
  st->fin = st->nimf >= K;
  st->action = kEndImf;
  if (st->fin) st->active = 0;
}

// One workgroup per signal: carries and ranks across its tiles, knot totals,
// and the step's action (Sec. 2.1 Step 5):
//   last step's sift met the SD criterion  -> kEndImf
//   siftable candidate, sift < S-1  -> kSift
//   siftable candidate, sift = S-1  -> kSiftLast (the IMF ends after it)
//   not siftable, sift > 0          -> kEndImf   (the candidate is the IMF)
//   not siftable, sift = 0          -> kFinish   (the residue is final)
// An IMF end that reaches K IMFs also finishes the decomposition.
__global__ void __launch_bounds__(kTT) st_scan_kernel(const StreamSig* __restrict__ sigs) {
  __shared__ int64_t scratch64[kNW];
  __shared__ int scratch[kNW];
  __shared__ double wsum[2 * kNW];
  const StreamSig& S = sigs[blockIdx.x];
  SigStatus* st = S.st;
  if (S.trace && threadIdx.x == 0) st->tr_rec = -1;  // no detection record (yet)
  if (!st->active) {
    if (threadIdx.x == 0) st->action = kIdle;
    return;
  }
  // a load or an IMF end left the IMF's first candidate in r only
  if (threadIdx.x == 0) st->in_r = st->action != kSift;
  const int nt = S.ntiles;
  if (S.sd > 0.0 && st->action == kSift) {
    // SD criterion over the whole signal: the tiles' sums of the last sift
    double num = 0.0, den = 0.0;
    for (int t = threadIdx.x; t < nt; t += kTT) {
      num += S.tinfo[t].sd_num;
      den += S.tinfo[t].sd_den;
    }
    double tnum, tden;
    block_sum2<kNW>(num, den, wsum, threadIdx.x & (kWave - 1), threadIdx.x / kWave, tnum, tden);
    if (tnum < S.sd * tden) {
      if (threadIdx.x == 0) end_imf(st, S.K);
      return;
    }
  }
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
      o.cont_knot = dmax | (dmin << 1);
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
    if (S.trace) {
      // the record's header; its positions are written by st_trace_kernel
      int32_t* T = S.trace;
      const int used = T[0], need = 4 + nmax + nmin;
      if (T[1] && used + need <= S.trace_cap) {
        T[used] = st->nimf;
        T[used + 1] = st->sift;
        T[used + 2] = nmax;
        T[used + 3] = nmin;
        T[0] = used + need;
        st->tr_rec = used;
        st->tr_n[0] = nmax;
        st->tr_n[1] = nmin;
      } else {
        T[1] = 0;
      }
    }
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
    if (action == kSiftLast || action == kEndImf) {
      end_imf(st, S.K);
      st->action = action;
      return;
    }
    if (action == kSift) st->sift += 1;
    else fin = 1;  // kFinish
    st->action = action;
    st->fin = fin;
    if (fin) st->active = 0;
  }
}

// One knot and its mirrored copies (Sec. 2.1 Step 2 with the mirror
// boundary): the knot list of one envelope is
//   [-k_P', ..., -k_1, k_1, ..., k_n, 2(L-1)-k_n, ..., 2(L-1)-k_{n-P'+1}],
// P' = min(2, n), mirrored knots carrying their source's value.
__device__ __forceinline__ void put_knot(global_ptr<int32_t> kt, global_ptr<double> ky, int g,
                                         int n, int L, int pos, double y) {
  const int Pp = n < 2 ? n : 2;
  kt[Pp + g] = pos;
  ky[Pp + g] = y;
  if (g < 2 || g >= n - 2) {
    const int hi = 2 * (L - 1);
    if (g == 0) { kt[Pp - 1] = -pos; ky[Pp - 1] = y; }
    if (g == 1 && Pp == 2) { kt[0] = -pos; ky[0] = y; }
    if (g == n - 1) { kt[Pp + n] = hi - pos; ky[Pp + n] = y; }
    if (g == n - 2 && Pp == 2) { kt[Pp + n + 1] = hi - pos; ky[Pp + n + 1] = y; }
  }
}

// The knots of the tile at their ranks (Sec. 2.1 Step 1 -> Step 2): the
// continued run's extremum, when the scan found one, then the tile's own
// knots as detection listed them.  Also the tile's edge samples before this
// step (and, when the step ends the IMF, the residue's), for the evaluation
// of the neighbouring tiles.  One wave per tile (kCompactWaves tiles per
// workgroup, independent of each other): a tile holds a few hundred knots
// at most, and the time of a launch over every tile of a batch goes to each
// tile's chain of dependent descriptor reads, so more tiles in flight is
// what counts.
__global__ void __launch_bounds__(kCompactThreads) st_compact_kernel(
    const StreamSig* __restrict__ sigs, const int2* __restrict__ tiles, int ntiles) {
  // (the wave index read as wave-uniform: the tile's descriptor fields then
  // live in scalar registers)
  const int64_t tix = (int64_t)blockIdx.x * kCompactWaves +
                      __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (tix >= ntiles) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int2 tv = tiles[tix];
  const StreamSig& S = sigs[tv.x];
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  const int64_t lo = (int64_t)tv.y * kTileKnots;
  // The status, the tile's counts and ranks, the first list entries and the
  // edge samples are read together, before the status decides whether the
  // tile has work: a chain of dependent reads is what a launch over every
  // tile of a batch waits on.  (All of them lie in the signal's buffers
  // whatever the step.)
  const global_ptr<const SigStatus> st = gmem<const SigStatus>(S.st);
  const auto& ti = gmem<const TileInfo>(S.tinfo)[tv.y];
  const int action = st->action, in_r = st->in_r, nk[2] = {st->n[0], st->n[1]};
  const int cnt[2] = {ti.cnt[0], ti.cnt[1]}, off[2] = {ti.off[0], ti.off[1]};
  const int cont_knot = ti.cont_knot;
  int p0[2];
  double v0[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    p0[e] = gmem<const int32_t>(S.lpos[e])[lo + lane];
    v0[e] = gmem<const double>(S.lval[e])[lo + lane];
  }
  double ea = 0.0, eb = 0.0;
  if (lane == 0) {
    const global_ptr<const double> hg = gmem<const double>(S.h);
    ea = hg[a];
    eb = hg[a + n - 1];
  }
  asm volatile("" ::"v"(p0[0]), "v"(p0[1]), "v"(v0[0]), "v"(v0[1]), "v"(ea), "v"(eb));
  if (action != kSift && action != kSiftLast && action != kEndImf) return;
  if (lane == 0) {
    // the residue's edge samples: the candidate's when it is in r, and, when
    // the step ends the IMF, for the new residue's detection
    double ra = 0.0, rb = 0.0;
    if (in_r || action != kSift) {
      const global_ptr<const double> rg = gmem<const double>(S.r);
      ra = rg[a];
      rb = rg[a + n - 1];
    }
    gmem(S.edge)[2 * tv.y] = in_r ? ra : ea;
    gmem(S.edge)[2 * tv.y + 1] = in_r ? rb : eb;
    if (action != kSift) {
      const global_ptr<double> re = gmem(S.edge) + 2 * (int64_t)S.ntiles;
      re[2 * tv.y] = ra;
      re[2 * tv.y + 1] = rb;
    }
  }
  if (action == kEndImf) return;  // no knots: the candidate is the IMF
  global_ptr<int32_t> kt[2];
  global_ptr<double> ky[2];
  global_ptr<const int32_t> lp[2];
  global_ptr<const double> lv[2];
  int ck[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    ck[e] = (cont_knot >> e) & 1;
    kt[e] = gmem(S.kt[e]);
    ky[e] = gmem(S.ky[e]);
    lp[e] = gmem<const int32_t>(S.lpos[e]) + lo;
    lv[e] = gmem<const double>(S.lval[e]) + lo;
    if (ck[e] && lane == 0)
      put_knot(kt[e], ky[e], off[e], nk[e], L, ((ti.carry >> 2) + ti.cont_pos) >> 1,
               ti.cont_y);
    if (lane < cnt[e]) put_knot(kt[e], ky[e], off[e] + ck[e] + lane, nk[e], L, p0[e], v0[e]);
  }
  // The rest of both lists in rounds of kCompactBatch entries per lane and
  // list, every round's loads issued before its stores: a dense tile holds
  // several hundred knots, and one load-store trip per entry would leave the
  // wave waiting on one load at a time.
  const int most = max(cnt[0], cnt[1]);
  for (int i0 = lane + kWave; i0 < most; i0 += kCompactBatch * kWave) {
    int p[2][kCompactBatch];
    double v[2][kCompactBatch];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int u = 0; u < kCompactBatch; ++u) {
        const int i = i0 + u * kWave;
        if (i < cnt[e]) {
          p[e][u] = lp[e][i];
          v[e][u] = lv[e][i];
        }
      }
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int u = 0; u < kCompactBatch; ++u) {
        const int i = i0 + u * kWave;
        if (i < cnt[e]) put_knot(kt[e], ky[e], off[e] + ck[e] + i, nk[e], L, p[e][u], v[e][u]);
      }
  }
}

// The positions of this step's detection record (Sec. 2.1 Step 1), for the
// signals that carry a trace: the tile's extrema at the ranks the scan gave
// them, the continued run's extremum first, exactly as compaction places
// the knots (without the mirrored ones).
__global__ void __launch_bounds__(kTT) st_trace_kernel(const StreamSig* __restrict__ sigs,
                                                       const int2* __restrict__ tiles) {
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  if (!S.trace) return;
  const int rec = S.st->tr_rec;
  if (rec < 0) return;
  const TileInfo ti = S.tinfo[tv.y];
  const int64_t lo = (int64_t)tv.y * kTileKnots;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    int32_t* out = S.trace + rec + 4 + (e ? S.st->tr_n[0] : 0);
    const int ck = (ti.cont_knot >> e) & 1;
    if (ck && threadIdx.x == 0) out[ti.off[e]] = ((ti.carry >> 2) + ti.cont_pos) >> 1;
    for (int i = threadIdx.x; i < ti.cnt[e]; i += kTT) out[ti.off[e] + ck + i] = S.lpos[e][lo + i];
  }
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------

// One block per (signal, envelope, kSB interior rows r0 .. r1-1): the knots
// of the block's window (its rows plus kHalo on each side, and their
// neighbours) are staged in LDS and the window's rows a0..a1 are solved
// exactly by the scans of the on-chip solver (each thread a stretch of R
// consecutive rows), started as if the rows beyond the window did not
// exist.  Windows that reach the ends of the system are exact; elsewhere the
// coupling a window drops is damped by at least (2 - sqrt 3)^kHalo at the
// block's own rows, because the matrix is symmetric with every diagonal
// twice its row's off-diagonal sum, so the Jacobi-scaled matrix has
// condition number at most 3 and an inverse whose entries decay
// geometrically at that rate.  Each thread writes the second derivatives
// m_j of its rows in r0..r1-1, and the zeros of the two end knots when it
// holds row 1 or row n-2; the evaluation forms each segment's cubic from
// the knots at its ends.
// (bounded to 72 VGPRs, which it fits without spilling: seven waves per
// SIMD; the LDS window would allow eight workgroups per CU)
__global__ void __launch_bounds__(kTT, 7) st_solve_kernel(const StreamSig* __restrict__ sigs,
                                                          const int4* __restrict__ blocks) {
  constexpr int kW = kSB + 2 * kHalo + 4;
  constexpr int kRMax = (kSB + 2 * kHalo + kTT - 1) / kTT;
  __shared__ int32_t lt[kW];
  __shared__ double ly[kW];
  __shared__ __align__(16) double fwd_lds[kFwdStride * kNW];
  __shared__ double bwd_lds[2 * kNW];
  const int4 bv = blocks[blockIdx.x];  // (signal, envelope, first block, stride)
  const StreamSig& S = sigs[bv.x];
  if (!sifting(*S.st)) return;
  const int env = bv.y;
  const int n = S.st->n[env];
  const int Pp = n < 2 ? n : 2;
  const int n2 = n + 2 * Pp;
  // this workgroup's blocks: bv.z, bv.z + G, ... (G = bv.w workgroups per
  // envelope)
  const int nbt = solve_blocks(S.cap), G = max(bv.w, 1);
  for (int blk = bv.z; blk < nbt; blk += G) {
    const int r0 = 1 + blk * kSB;
    if (n2 < 3 || r0 > n2 - 2) break;
    if (blk != bv.z) __syncthreads();  // the previous block is done with the LDS
    const int r1 = min(r0 + kSB, n2 - 1);  // rows r0 .. r1-1
    const int a0 = max(1, r0 - kHalo), a1 = min(n2 - 2, r1 - 1 + kHalo);
    const int w0 = a0 - 1, w1 = a1 + 1;    // knots read
    const global_ptr<const int32_t> kt = gmem<const int32_t>(S.kt[env]);
    const global_ptr<const double> ky = gmem<const double>(S.ky[env]);
    {
      // knot pairs from an even index (16-byte value loads), the window's
      // first knot alone when w0 is odd and its last when a pair is left
      const int nw = w1 - w0 + 1, head = w0 & 1, np = (nw - head) / 2;
      const global_ptr<const RankPair> t2 = (global_ptr<const RankPair>)(kt + w0 + head);
      const global_ptr<const SamplePair> y2 = (global_ptr<const SamplePair>)(ky + w0 + head);
      for (int p = threadIdx.x; p < np; p += kTT) {
        const auto& tp = t2[p];
        const auto& yp = y2[p];
        const int32_t ta = tp.x, tb = tp.y;
        const double ya = yp.x, yb = yp.y;
        const int i = head + 2 * p;
        lt[i] = ta;
        lt[i + 1] = tb;
        ly[i] = ya;
        ly[i + 1] = yb;
      }
      if (threadIdx.x == 0 && head) {
        lt[0] = kt[w0];
        ly[0] = ky[w0];
      }
      if (threadIdx.x == kWave && ((nw - head) & 1)) {
        lt[nw - 1] = kt[w1];
        ly[nw - 1] = ky[w1];
      }
    }
    __syncthreads();
  #define T(j) ((double)lt[(j) - w0])
  #define Y(j) (ly[(j) - w0])
    const int rows = a1 - a0 + 1;
    // (<= kRMax; a multiple of 4 is raised by one: row blocks whose starts
    // lie a multiple of 8 doubles apart would share LDS banks 4 ways or more)
    int R = (rows + kTT - 1) / kTT;
    R += (R & 3) == 0 ? 1 : 0;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int j0 = a0 + threadIdx.x * R;
    // row j's equation a M_{j-1} + b M_j + c M_{j+1} = r; sl brings in the
    // slope of segment j-1 and takes out that of segment j (a thread's
    // consecutive rows share a segment's slope: one reciprocal per row)
    auto row = [&](int j, double& sl, double& a, double& b, double& c, double& r) {
      const double tm = T(j - 1), t0 = T(j), tp = T(j + 1);
      a = t0 - tm;
      c = tp - t0;
      b = 2.0 * (a + c);
      const double sn = (Y(j + 1) - Y(j)) * recip(c);
      r = 6.0 * (sn - sl);
      sl = sn;
    };
    // the slope of segment j-1, which enters row j
    auto slope_into = [&](int j) { return (Y(j) - Y(j - 1)) * recip(T(j) - T(j - 1)); };
    FwdMap G = fwd_identity();
    double sl = j0 <= a1 ? slope_into(j0) : 0.0;
  #pragma unroll
    for (int q = 0; q < kRMax; ++q) {
      const int j = j0 + q;
      if (q < R && j <= a1) {
        double a, b, c, r;
        row(j, sl, a, b, c, r);
        G = fwd_row_after(a, b, c, r, G);
        if ((q & 3) == 3) fwd_normalize(G);
      }
    }
    fwd_normalize(G);
    G = fwd_wave_scan(G);
    if (lane == kWave - 1) {
      double* o = fwd_lds + kFwdStride * wid;
      o[0] = G.a00; o[1] = G.a01; o[2] = G.a10; o[3] = G.a11;
      o[4] = G.v0; o[5] = G.v1; o[6] = G.s;
    }
    __syncthreads();
    double cpa[kRMax], dpa[kRMax];
    {
      double Q, P, D;
      fwd_enter(fwd_lds, wid, Q, P, D);
      const FwdMap Y1 = fwd_dpp<kDppWaveShr1, 0xf>(G);
      if (lane > 0) {
        fwd_apply(Y1, Q, P, D);
        vec_normalize(Q, P, D);
      }
      double sl2 = j0 <= a1 ? slope_into(j0) : 0.0;
  #pragma unroll
      for (int q = 0; q < kRMax; ++q) {
        cpa[q] = 0.0;
        dpa[q] = 0.0;
        const int j = j0 + q;
        if (q < R && j <= a1) {
          double a, b, c, r;
          row(j, sl2, a, b, c, r);
          const double qn = fma(b, Q, -a * P);
          D = fma(r, Q, -a * D);
          P = c * Q;
          Q = qn;
          vec_normalize(Q, P, D);
          const double iq = recip(Q);
          cpa[q] = P * iq;
          dpa[q] = D * iq;
        }
      }
    }
    // back-substitution maps composed from the thread's last row down
    double al = 0.0, be = 1.0;
  #pragma unroll
    for (int q = kRMax - 1; q >= 0; --q) {
      if (q < R && j0 + q <= a1) {
        al = fma(-cpa[q], al, dpa[q]);
        be = -cpa[q] * be;
      }
    }
    bwd_wave_scan<false>(al, be, lane);  // (the fill raises this kernel's registers)
    if (lane == 0) {
      bwd_lds[2 * wid] = al;
      bwd_lds[2 * wid + 1] = be;
    }
    __syncthreads();
    double Mn = bwd_after(bwd_lds, wid, kNW);
    {
      const double a2 = dpp_move<kDppWaveShl1, 0xf>(al), b2 = dpp_move<kDppWaveShl1, 0xf>(be);
      if (lane + 1 < kWave) Mn = fma(b2, Mn, a2);
    }
    // The block's second derivatives go through the LDS window (its values
    // are no longer read: every thread is past the forward passes) and out
    // in coalesced stores; a thread's own rows lie R doubles apart from its
    // neighbours'.
  #pragma unroll
    for (int q = kRMax - 1; q >= 0; --q) {
      const int j = j0 + q;
      if (q < R && j <= a1) {
        const double Mj = fma(-cpa[q], Mn, dpa[q]);
        if (j >= r0 && j < r1) ly[j - w0] = Mj;
        Mn = Mj;
      }
    }
    __syncthreads();
    const global_ptr<double> km = gmem(S.km[env]);
    for (int j = r0 + threadIdx.x; j < r1; j += kTT) km[j] = ly[j - w0];
    if (threadIdx.x == 0) {  // natural end conditions
      if (r0 == 1) km[0] = 0.0;
      if (r1 == n2 - 1) km[n2 - 1] = 0.0;
    }
  }
#undef T
#undef Y
}

// Walker over the segments of one envelope of a streaming signal, reading
// the knots (position, value, second derivative) in global memory: the
// current segment j = [t0, t1), its right knot (t1, y1, m1), its halved
// power-form coefficients and B = k - t0.  On [t_j, t_{j+1}), with
// B = k - t_j and g = t_{j+1} - t_j, the natural spline is
//   y_j + b_j B + (m_j / 2) B^2 + ((m_{j+1} - m_j) / (6 g)) B^3,
//   b_j = (y_{j+1} - y_j) / g - g (2 m_j + m_{j+1}) / 6,
// and the walker evaluates half of it (the envelope mean is the sum of two
// halves).  (Waves whose segments fit one per lane take the wave-shared walk
// in st_eval_kernel instead; this walker serves the denser ones.)
struct StWalk {
  int j, t1;
  double y1, m1, B, q0, q1, q2, q3;
};

// One envelope's knots (positions, values, second derivatives) in global
// memory, and the index of its last knot.
struct KnotView {
  global_ptr<const int32_t> t;
  global_ptr<const double> y, m;
  int last;
};

__device__ __forceinline__ KnotView knot_view(const StreamSig& S, int e, int nk) {
  const int Pp = nk < 2 ? nk : 2;
  return {gmem<const int32_t>(S.kt[e]), gmem<const double>(S.ky[e]),
          gmem<const double>(S.km[e]), nk + 2 * Pp - 1};
}

// The coefficients of segment j from its left knot (t0, y0, m0) and the
// right knot (w.t1, w.y1, w.m1).
__device__ __forceinline__ void st_walk_coefs(StWalk& w, int j, int t0, double y0, double m0) {
  w.j = j;
  const double g = (double)(w.t1 - t0);
  const double ig = recip(g);
  const double b = (w.y1 - y0) * ig - g * fma(2.0, m0, w.m1) * (1.0 / 6.0);
  w.q0 = 0.5 * y0;
  w.q1 = 0.5 * b;
  w.q2 = 0.25 * m0;
  w.q3 = (w.m1 - m0) * ig * (1.0 / 12.0);
}

// The segment holding sample k, searched forward from segment j (whose left
// knot lies at or before k; the last knot lies beyond the signal), and its
// left knot's position t0.
__device__ __forceinline__ int st_walk_find(const KnotView& K, int j, int k, int& t0) {
  t0 = K.t[j];
  int t1 = K.t[j + 1];
  while (t1 <= k) {
    ++j;
    t0 = t1;
    t1 = K.t[j + 1];
  }
  return j;
}

// A walker on segment j, at sample k.
__device__ __forceinline__ void st_walk_init(StWalk& w, const KnotView& K, int j, int k) {
  const int t0 = K.t[j];
  w.t1 = K.t[j + 1];
  w.y1 = K.y[j + 1];
  w.m1 = K.m[j + 1];
  st_walk_coefs(w, j, t0, K.y[j], K.m[j]);
  w.B = (double)(k - t0);
}

// A segment's halved power-form coefficients and its right knot's
// position, as one lane of a wave holds them for the others (the
// wave-shared walk).
struct SegCoefs {
  double q0, q1, q2, q3;
  int t1;
};

// Segment j's coefficients, formed as a walker forms them at a crossing.
__device__ __forceinline__ SegCoefs seg_coefs(const KnotView& K, int j) {
  StWalk w;
  const int t0 = K.t[j];
  w.t1 = K.t[j + 1];
  w.y1 = K.y[j + 1];
  w.m1 = K.m[j + 1];
  st_walk_coefs(w, j, t0, K.y[j], K.m[j]);
  return {w.q0, w.q1, w.q2, w.q3, w.t1};
}

// Lane `src`'s segment (every lane of the wave active).
__device__ __forceinline__ SegCoefs seg_from_lane(const SegCoefs& own, int src) {
  return {__shfl(own.q0, src), __shfl(own.q1, src), __shfl(own.q2, src), __shfl(own.q3, src),
          __shfl(own.t1, src)};
}

// Half the envelope at sample k (one step from k-1 crosses at most one knot).
__device__ __forceinline__ double st_walk_at(StWalk& w, const KnotView& K, int k) {
  if (w.t1 <= k) {
    const int t0 = w.t1;
    const double y0 = w.y1, m0 = w.m1;
    w.B = (double)(k - t0);
    w.t1 = K.t[w.j + 2];
    w.y1 = K.y[w.j + 2];
    w.m1 = K.m[w.j + 2];
    st_walk_coefs(w, w.j + 1, t0, y0, m0);
  }
  return fma(fma(fma(w.q3, w.B, w.q2), w.B, w.q1), w.B, w.q0);
}

// ---------------------------------------------------------------------------
// Evaluate and update
// ---------------------------------------------------------------------------

// One step's work on the tile's samples:
//   kSift, kSiftLast  envelope means removed (Sec. 2.1 Steps 2-4): each
//                     thread walks the knots covering its samples, starting
//                     from its rank (detection's in-tile ranks plus the
//                     scan's tile offsets);
//   kSiftLast, kEndImf  IMF end: the candidate is stored in its output slot
//                     (deserialized, Sec. 3.3), r <- r - h, and r is the
//                     next step's candidate (h is not written);
//   final             residue into slot K, unused IMF slots zero (Sec. 4.3),
//                     IMF count and statistics.
//
// SD: some signal of the launch stops its IMFs by the SD rule, whose sums
// the sift accumulates; the instance without them holds fewer registers
// through the walk.
template <bool SD>
__global__ void __launch_bounds__(kTT, 8) st_eval_kernel(const StreamSig* __restrict__ sigs,
                                                      const int2* __restrict__ tiles) {
  __shared__ double tbuf[kTile];
  __shared__ int pub_key[kTT];
  __shared__ int scratch[kNW];
  __shared__ int64_t scratch64[kNW];
  __shared__ double halo[2];  // the neighbours' edge samples after the sift
  __shared__ double wsum[2 * kNW];
  __shared__ int cont_exit, cont_pos;
  __shared__ double cont_y;
  const int2 tv = tiles[blockIdx.x];
  const StreamSig& S = sigs[tv.x];
  const global_ptr<const SigStatus> st = gmem<const SigStatus>(S.st);
  const int action = st->action;
  if (action == kIdle) return;
  const int L = S.L;
  const int a = tv.y * kTile, n = min(kTile, L - a);
  const global_ptr<double> hg = gmem(S.h);
  // The candidate tile's sample pairs are loaded into registers first, and
  // stored to the tile buffer only after the walk's start below has issued
  // its own reads (ranks, tile counts, knot positions), so that the two
  // latencies overlap.  Pairs are 16-byte loads (a tile starts at an even
  // sample of a 256-byte-aligned buffer); samples 2j and 2j+1 land at
  // tsw(2j) and tsw(2j) ^ 1.
  constexpr int kPairs = kTile / 2 / kTT;
  static_assert(kPairs * 2 * kTT == kTile, "a tile is whole pairs per thread");
  double px[kPairs], py[kPairs];
  double odd = 0.0;
  {
    const global_ptr<const double> cand = st->in_r ? gmem<const double>(S.r) : hg;
    const global_ptr<const SamplePair> c2 = (global_ptr<const SamplePair>)(cand + a);
#pragma unroll
    for (int u = 0; u < kPairs; ++u) {
      const int j = threadIdx.x + u * kTT;
      if (j < n / 2) {
        const auto& v = c2[j];  // (one 16-byte load)
        px[u] = v.x;
        py[u] = v.y;
      }
    }
    if ((n & 1) && threadIdx.x == 0) odd = cand[a + n - 1];
  }
  const bool sift = action == kSift || action == kSiftLast;
  const int lb = threadIdx.x * kTC;
  const int nv = max(0, min(kTC, n - lb));
  const int k0 = a + lb;
  // thread 0 starts one sample early for the previous tile's last sample
  const int ks = (threadIdx.x == 0 && a > 0) ? k0 - 1 : k0;
  const KnotView kv[2] = {knot_view(S, 0, st->n[0]), knot_view(S, 1, st->n[1])};
  // the thread holding the tile's last sample continues to the next tile's
  // first sample
  const bool tail = nv > 0 && lb + nv == n && a + n < L;
  int js[2] = {0, 0}, jt0[2] = {0, 0};  // the segments holding sample ks, their left knots
  if (sift && nv > 0) {
    const uint32_t tr =
        (uint32_t)gmem<const int32_t>(S.trank)[(int64_t)tv.y * kTT + threadIdx.x];
    const auto& ti = gmem<const TileInfo>(S.tinfo)[tv.y];
    // the continued run's extremum precedes this thread's knots when the
    // run ends in an earlier thread of the tile
    const bool cont_before = ti.cont_pos >= 0 && ti.cont_pos < k0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int nk = st->n[e];
      const int Pp = nk < 2 ? nk : 2;
      const int rank = ti.off[e] + (cont_before ? ((ti.cont_knot >> e) & 1) : 0) +
                       (int)(e ? tr >> 16 : tr & 0xffffu);
      // the last knot of earlier threads lies before the thread's first
      // sample (and before sample a-1 for thread 0: it lies in an earlier
      // tile or is a mirrored knot)
      js[e] = st_walk_find(kv[e], Pp + rank - 1, ks, jt0[e]);
    }
  }
#pragma unroll
  for (int u = 0; u < kPairs; ++u) {
    const int j = threadIdx.x + u * kTT;
    if (j < n / 2) {
      const int s0 = tsw(2 * j);
      tbuf[s0] = px[u];
      tbuf[s0 ^ 1] = py[u];
    }
  }
  if ((n & 1) && threadIdx.x == 0) tbuf[tsw(n - 1)] = odd;
  if (sift) {
    if (threadIdx.x == 0) cont_exit = 0;
    __syncthreads();
    double num = 0.0, den = 0.0;  // the tile's sums for the SD criterion
    // The wave-shared walk: when the segments the wave's samples fall in
    // number at most 64 for each envelope, lane i forms the coefficients of
    // the wave's i-th segment once, and a lane that crosses a knot takes its
    // new segment from the lane holding it.  A wave runs the crossing code
    // at a sample whenever any of its lanes crosses there; this way that
    // code is a few lane exchanges instead of the coefficients' arithmetic.
    // A lane's samples k0 .. k0+kTC (with the tail sample) hold at most 5
    // knots of an envelope (knots of one envelope lie at least two samples
    // apart).  The arithmetic is the walkers', value for value.
    const unsigned long long live = __ballot(nv > 0);
    const int hi = live ? 63 - __clzll((long long)live) : 0;
    int J0[2], Jn[2];  // the wave's segments: J0 .. J0 + Jn - 1
    bool shared = live != 0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      J0[e] = __builtin_amdgcn_readfirstlane(js[e]);
      Jn[e] = __builtin_amdgcn_readlane(js[e], hi) + 6 - J0[e];
      shared = shared && Jn[e] <= kWave;
    }
    if (shared) {
      const int lane = threadIdx.x & (kWave - 1);
      SegCoefs own[2], cur[2];
      int sidx[2], t0[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        own[e] = lane < Jn[e] ? seg_coefs(kv[e], min(J0[e] + lane, kv[e].last - 1))
                              : SegCoefs{0.0, 0.0, 0.0, 0.0, 0};
        sidx[e] = js[e] - J0[e];
        cur[e] = seg_from_lane(own[e], sidx[e]);
        t0[e] = jt0[e];
      }
      // positions c = -1 (thread 0's sample a-1), 0 .. nv-1 (the thread's
      // samples), nv (the tail sample)
#pragma unroll
      for (int c = -1; c <= kTC; ++c) {
        const int k = k0 + c;
        const bool act = c < 0 ? ks < k0 : (c < nv || (c == nv && tail));
        double m = 0.0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const bool cross = act && cur[e].t1 <= k;
          if (__any(cross)) {
            if (cross) t0[e] = cur[e].t1;  // the new segment starts at the old one's end
            sidx[e] += cross ? 1 : 0;
            cur[e] = seg_from_lane(own[e], sidx[e]);
          }
          const double B = (double)(k - t0[e]);
          const double v = fma(fma(fma(cur[e].q3, B, cur[e].q2), B, cur[e].q1), B, cur[e].q0);
          m = e == 0 ? v : m + v;
        }
        if (act) {
          if (c < 0) {
            halo[0] = gmem(S.edge)[2 * tv.y - 1] - m;
          } else if (c < nv) {
            const double hk = tbuf[tsw(lb + c)];
            if constexpr (SD) {
              num = fma(m, m, num);
              den = fma(hk, hk, den);
            }
            tbuf[tsw(lb + c)] = hk - m;
          } else {
            halo[1] = gmem(S.edge)[2 * tv.y + 2] - m;
          }
        }
      }
    } else if (nv > 0) {
      StWalk wk[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) st_walk_init(wk[e], kv[e], js[e], ks);
      if (ks < k0) {
        const double up = st_walk_at(wk[0], kv[0], ks);
        const double lo = st_walk_at(wk[1], kv[1], ks);
        halo[0] = gmem(S.edge)[2 * tv.y - 1] - (up + lo);
        wk[0].B += 1.0;
        wk[1].B += 1.0;
      }
#pragma unroll
      for (int c = 0; c < kTC; ++c) {
        if (c < nv) {
          const int k = k0 + c;
          const double up = st_walk_at(wk[0], kv[0], k);
          const double lo = st_walk_at(wk[1], kv[1], k);
          const double m = up + lo, hk = tbuf[tsw(lb + c)];
          if constexpr (SD) {
            num = fma(m, m, num);
            den = fma(hk, hk, den);
          }
          tbuf[tsw(lb + c)] = hk - m;
          wk[0].B += 1.0;
          wk[1].B += 1.0;
        }
      }
      if (tail) {
        const int k = a + n;
        const double up = st_walk_at(wk[0], kv[0], k);
        const double lo = st_walk_at(wk[1], kv[1], k);
        halo[1] = gmem(S.edge)[2 * tv.y + 2] - (up + lo);
      }
    }
    if (action == kSift && SD && S.sd > 0.0) {
      double tnum, tden;
      block_sum2<kNW>(num, den, wsum, threadIdx.x & (kWave - 1), threadIdx.x / kWave, tnum,
                      tden);
      if (threadIdx.x == 0) {
        gmem(S.tinfo)[tv.y].sd_num = tnum;
        gmem(S.tinfo)[tv.y].sd_den = tden;
      }
    }
  }
  __syncthreads();
  const int64_t M = S.M, R = S.M + S.D;
  if (action == kSiftLast || action == kEndImf) {
    const global_ptr<double> slot = gmem(S.out) + (int64_t)st->slot * S.slot_stride;
    const global_ptr<double> rg = gmem(S.r);
    // all of the thread's residue samples are loaded before any store (the
    // compiler cannot move a load above a store to the output, which might
    // alias it)
    double rv[kTC];
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int i = threadIdx.x + c * kTT;
      rv[c] = i < n ? rg[a + i] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kTC; ++c) {
      const int i = threadIdx.x + c * kTT;
      if (i < n) {
        const int k = a + i;
        const double hk = tbuf[tsw(i)];
        const double nr = rv[c] - hk;
        rg[k] = nr;
        tbuf[tsw(i)] = nr;
        const int64_t ii = k / R, m = k - ii * R;
        if (m < M) slot[ii * M + m] = hk;
      }
    }
  }
  // The next step's candidate is on chip now: the sifted candidate (kSift),
  // or the next IMF's first candidate h = r after an IMF end.  Its extrema
  // are detected here, so a step starts with its candidate's extrema known.
  // The neighbours' edge samples of a new residue are their residue before
  // this step (kept by compaction) less their candidate (sifted by the walk
  // under kSiftLast, as compaction kept it under kEndImf).
  const bool fin = st->fin;
  const bool detect = !fin;  // (kSift never finishes)
  if (detect) {
    if (action != kSift) {
      const global_ptr<const double> eg = gmem<const double>(S.edge);
      const global_ptr<const double> re = eg + 2 * (int64_t)S.ntiles;
      if (threadIdx.x == 0) {
        cont_exit = 0;
        if (a > 0) halo[0] = re[2 * tv.y - 1] - (action == kEndImf ? eg[2 * tv.y - 1] : halo[0]);
      }
      if (threadIdx.x == kWave && a + n < L)
        halo[1] = re[2 * tv.y + 2] - (action == kEndImf ? eg[2 * tv.y + 2] : halo[1]);
      __syncthreads();
    }
    const double prev = a > 0 ? halo[0] : 0.0;
    const double next = a + n < L ? halo[1] : 0.0;
    const int first_key =
        a == 0 ? 0 : (prev != tbuf[tsw(0)] ? a * 4 + step_kind(prev, tbuf[tsw(0)]) : kCont);
    const int lb = threadIdx.x * kTC;
    double h[kTC];
#pragma unroll
    for (int c = 0; c < kTC; ++c) h[c] = lb + c < n ? tbuf[tsw(lb + c)] : 0.0;
    TileDet d;
    tile_detect<kTC>(h, a, n, L, threadIdx.x, first_key, next, tbuf, pub_key,
                     &cont_exit, &cont_pos, &cont_y, d);
    __syncthreads();
    // the sifted candidate goes out now (a new IMF's first candidate is in r
    // already); the tile buffer then stages the knot lists
    if (action == kSift)
      store_tile(hg + a, n, tbuf);
    record_tile(d, h, a, first_key, cont_exit, cont_pos, cont_y, S, tv.y, scratch64, scratch,
                tbuf);
  }
  if (fin) {
    const int K = S.K, bad = st->bad;
    const int nimf = bad ? 0 : st->nimf;
    for (int i = threadIdx.x; i < n; i += kTT) {
      const int k = a + i;
      const int64_t ii = k / R, m = k - ii * R;
      if (m < M) {
        const int64_t o = ii * M + m;
        const global_ptr<double> og = gmem(S.out);
        for (int q = nimf; q < K; ++q) og[q * S.slot_stride + o] = 0.0;
        og[(int64_t)K * S.slot_stride + o] = bad ? 0.0 : tbuf[tsw(i)];
      }
    }
    if (tv.y == 0 && threadIdx.x == 0) {
      if (S.n_imfs) *S.n_imfs = bad ? -5 : nimf;
      if (S.stats) {
        S.stats[0] = st->n_sifts;
        S.stats[1] = st->n_knots;
        S.stats[2] = st->n_sifts * (int64_t)S.L;
      }
      gmem(S.st)->done = 1;
    }
  }
}

__global__ void st_gather_done_kernel(const StreamSig* __restrict__ sigs, int n,
                                      int32_t* __restrict__ done) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) done[i] = sigs[i].st->done;
}

// The descriptor of one signal and its tables, as stream_tables() lays them
// out for a one-signal batch: tiles[t] = (0, t) and blocks[e * nb + z] =
// (0, e, z, nb) for the envelopes e = 0, 1 and their solve workgroups z < nb.
__global__ void st_put_single_kernel(StreamSig g, StreamSig* __restrict__ dsig,
                                     int2* __restrict__ tiles, int ntiles,
                                     int4* __restrict__ blocks, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *dsig = g;
  if (i == 0 && g.trace) {
    g.trace[0] = 4;  // entries used: the header
    g.trace[1] = 1;  // every record fitted
    g.trace[2] = 0;
    g.trace[3] = 0;
  }
  if (i < ntiles) tiles[i] = make_int2(0, i);
  if (i < 2 * nb) blocks[i] = make_int4(0, i / nb, i - (i / nb) * nb, nb);
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
                   const int4* blocks, int nblocks, hipStream_t st, bool sd, bool trace,
                   const hipEvent_t* marks) {
  if (nsig <= 0) return hipSuccess;
  auto mark = [&](int i) { if (marks) (void)hipEventRecord(marks[i], st); };
  mark(0);
  hipLaunchKernelGGL(st_scan_kernel, dim3(nsig), dim3(kTT), 0, st, sigs);
  if (trace) hipLaunchKernelGGL(st_trace_kernel, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  mark(1);
  hipLaunchKernelGGL(st_compact_kernel, dim3((ntiles + kCompactWaves - 1) / kCompactWaves),
                     dim3(kCompactThreads), 0, st, sigs, tiles, ntiles);
  mark(2);
  hipLaunchKernelGGL(st_solve_kernel, dim3(nblocks), dim3(kTT), 0, st, sigs, blocks);
  mark(3);
  if (sd)
    hipLaunchKernelGGL(st_eval_kernel<true>, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  else
    hipLaunchKernelGGL(st_eval_kernel<false>, dim3(ntiles), dim3(kTT), 0, st, sigs, tiles);
  mark(4);
  return hipGetLastError();
}
hipError_t st_put_single(const StreamSig& g, StreamSig* dsig, int2* tiles, int4* blocks,
                         hipStream_t s) {
  const int nb = stream_solve_groups(g.cap, stream_solve_fold(2 * stream_solve_blocks(g.cap)));
  const int n = g.ntiles > 2 * nb ? g.ntiles : (2 * nb > 1 ? 2 * nb : 1);
  hipLaunchKernelGGL(st_put_single_kernel, dim3((n + 255) / 256), dim3(256), 0, s, g, dsig,
                     tiles, g.ntiles, blocks, nb);
  return hipGetLastError();
}
hipError_t st_gather_done(const StreamSig* sigs, int nsig, int32_t* done, hipStream_t s) {
  if (nsig <= 0) return hipSuccess;
  hipLaunchKernelGGL(st_gather_done_kernel, per_signal(nsig), dim3(256), 0, s, sigs, nsig, done);
  return hipGetLastError();
}

int stream_solve_blocks(int cap) { return solve_blocks(cap); }

int stream_solve_fold(int64_t total_blocks, int target) {
  return launch_fold(total_blocks, target > 0 ? target : kSolveTarget);
}

int stream_solve_groups(int cap, int fold) {
  return (stream_solve_blocks(cap) + fold - 1) / fold;
}

}  // namespace semd
