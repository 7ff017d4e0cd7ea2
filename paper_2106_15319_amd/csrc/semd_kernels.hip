// HIP kernels of the Serial-EMD hot path for gfx950 (MI355X), FP64 throughout.
//
// Resident path: one workgroup decomposes one serialized signal (or one EEMD
// or CEEMDAN realization) completely on chip.  The candidate h lives in
// registers in a blocked layout (thread t owns samples [t*C, t*C + C)); the
// knots of the envelopes, their spline second derivatives and segment
// coefficients live in LDS; the residue r is read and written once per IMF.
// Per sift:
//   extrema (Sec. 2.1 Step 1)   neighbour exchange through LDS, plateau runs
//                                resolved by a walk over published run starts,
//                                per-thread counts, one block scan (wave
//                                shuffles + LDS wave totals) for compaction;
//   envelopes (Step 2)           each thread writes its own knots, a few the
//                                mirrored end knots; natural-spline second
//                                derivatives by two block-wide scans (forward
//                                elimination maps, then back-substitution);
//                                evaluation by a per-thread walk over segments;
//   mean and update (Steps 3-4)  fused into the evaluation.
// Serialization (Sec. 3.2) and the ensemble noise (Sec. 2.2) are fused into
// the first load; deserialization (Sec. 3.3) into the IMF and residue stores.
// The file also holds the single-step kernels and the CEEMDAN stage kernels.
#include <algorithm>

#include "semd_device.h"

namespace semd {
namespace {

using namespace dev;


// ---------------------------------------------------------------------------
// Resident-path building blocks (blocked layout: thread t owns the C samples
// [t*C, t*C + C) of the signal in registers h[])
// ---------------------------------------------------------------------------

// Knot store of the envelopes of one sift.  Knot j holds abscissa t_j and
// value y_j; the solve (solve_envelopes) leaves the halved power-form
// coefficients of segment [t_j, t_{j+1}) that the walker reads: y_j / 2 in y,
// m_j / 4 in m (m_j the spline second derivative), and the linear and cubic
// coefficients in q1 and q3.  34 bytes per knot.
struct Knots {
  double* y;
  double* m;
  double* q1;
  double* q3;
  int16_t* t;
};

constexpr int kKnotBytes = 4 * (int)sizeof(double) + (int)sizeof(int16_t);

// A store of cap knots in the region p.
__device__ __forceinline__ Knots knots_in(unsigned char* p, int cap) {
  Knots s;
  s.y = reinterpret_cast<double*>(p);
  s.m = s.y + cap;
  s.q1 = s.m + cap;
  s.q3 = s.q1 + cap;
  s.t = reinterpret_cast<int16_t*>(s.q3 + cap);
  return s;
}

__device__ __forceinline__ Knots knots_from(const Knots& a, int o) {
  Knots s;
  s.y = a.y + o;
  s.m = a.m + o;
  s.q1 = a.q1 + o;
  s.q3 = a.q3 + o;
  s.t = a.t + o;
  return s;
}

// Extrema of the candidate (Sec. 2.1 Step 1) from per-thread step masks.
// Bit b of R (F) is set when sample b of the thread is above (below) sample
// b-1; bit 0 compares with the previous thread's last sample and bit C with
// the next thread's first, so NE = R | F marks the starts of equal-valued
// runs.  A sample c closes a run when step c -> c+1 is not flat; the run is a
// maximum when it was entered rising and is left falling (minimum: the
// reverse), and its knot sits at the floor-middle of the run.  A run that
// starts in an earlier thread takes its entry kind from `carry` (key
// 4*start + kind of the run holding the thread's first sample; kind 0 for the
// run that starts at sample 0, which is never an extremum).  Contains one
// barrier.
template <int NT, int C>
__device__ __forceinline__ void rd_detect(const double (&h)[C], int base, int nv, int L, int tid,
                                          double* pub_first, double* pub_last, int* pub_key,
                                          unsigned& R, unsigned& F, int& carry,
                                          unsigned& maxbits, unsigned& minbits) {
  // step bits b = C-1 .. 1 shifted in from the top (doubling plus the
  // comparison: one add with carry each), then the bits of samples beyond
  // nv cleared
  R = 0u;
  F = 0u;
#pragma unroll
  for (int b = C - 1; b >= 1; --b) {
    R = R + R + (h[b] > h[b - 1] ? 1u : 0u);
    F = F + F + (h[b] < h[b - 1] ? 1u : 0u);
  }
  const unsigned live = nv > 0 ? (1u << nv) - 1u : 0u;
  R = (R << 1) & live;
  F = (F << 1) & live;
  if (nv > 0) {
    const unsigned inner = R | F;
    int key = -1;
    if (inner) {
      const int b = 31 - __clz(inner);
      key = (base + b) * 4 + (((R >> b) & 1u) ? kRise : kFall);
    }
    double last = h[C - 1];
    if (nv < C) {
#pragma unroll
      for (int c = 0; c < C - 1; ++c)
        if (c == nv - 1) last = h[c];
    }
    pub_first[tid] = h[0];
    pub_last[tid] = last;
    pub_key[tid] = key;
  }
  __syncthreads();
  carry = 0;
  maxbits = 0u;
  minbits = 0u;
  if (nv <= 0) return;
  if (tid > 0) {
    const double prev = pub_last[tid - 1];
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
        if (tau == 0) { carry = 0; break; }
        const double pl = pub_last[tau - 1], pf = pub_first[tau];
        if (pl != pf) { carry = tau * C * 4 + step_kind(pl, pf); break; }
        --tau;
      }
    }
  }
  if (nv == C && base + C < L) {
    const double next = pub_first[tid + 1];
    R |= (next > h[C - 1] ? 1u : 0u) << C;
    F |= (next < h[C - 1] ? 1u : 0u) << C;
  }
  const unsigned NE = R | F;
  const unsigned valid = (1u << nv) - 1u;
  maxbits = R & (F >> 1) & valid;
  minbits = F & (R >> 1) & valid;
  // ends of runs longer than one sample (or holding the thread's first)
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
    // (both masks updated by value: a store through a selected reference
    // would keep them in scratch memory)
    const unsigned is_max = (kind == kRise && ((F >> (c + 1)) & 1u)) ? 1u : 0u;
    const unsigned is_min = (kind == kFall && ((R >> (c + 1)) & 1u)) ? 1u : 0u;
    maxbits |= is_max << c;
    minbits |= is_min << c;
  }
}

// Floor-middle of the equal-valued run that sample c of the thread closes.
__device__ __forceinline__ int run_mid(unsigned NE, int carry, int base, int c) {
  const unsigned below = NE & ((2u << c) - 1u);
  const int start = below ? base + (31 - __clz(below)) : (carry >> 2);
  return (start + base + c) >> 1;
}

// Write this thread's knots of one kind (bits) at ranks first.. among n,
// plus the mirrored end knots (Sec. 2.1 Step 2 with the mirror boundary):
//   [-k_P', ..., -k_1, k_1, ..., k_n, 2(L-1)-k_n, ..., 2(L-1)-k_{n-P'+1}],
// P' = min(2, n), mirrored knots carrying their source's value.
template <int C>
__device__ __forceinline__ void rd_emit(const double (&h)[C], unsigned bits, unsigned NE,
                                        int carry, int base, int L, int first, int n,
                                        const Knots ks) {
  const int Pp = n < 2 ? n : 2;
  const int hi = 2 * (L - 1);
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    if ((bits >> c) & 1u) {
      const int g = first + __popc(bits & ((1u << c) - 1u));
      const int mid = run_mid(NE, carry, base, c);
      const double y = h[c];
      ks.t[Pp + g] = (int16_t)mid;
      ks.y[Pp + g] = y;
      if (g < 2 || g >= n - 2) {
        if (g == 0) { ks.t[Pp - 1] = (int16_t)(-mid); ks.y[Pp - 1] = y; }
        if (g == 1 && Pp == 2) { ks.t[0] = (int16_t)(-mid); ks.y[0] = y; }
        if (g == n - 1) { ks.t[Pp + n] = (int16_t)(hi - mid); ks.y[Pp + n] = y; }
        if (g == n - 2 && Pp == 2) { ks.t[Pp + n + 1] = (int16_t)(hi - mid); ks.y[Pp + n + 1] = y; }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Natural-spline second derivatives and segment coefficients (Sec. 2.1
// Step 2) by two block-wide scans
// ---------------------------------------------------------------------------
//
// The knots of the sift's systems are taken as one sequence of rows k.  The
// first and last knot of each system read M_k = 0 (the natural end
// conditions); every other row reads
//   a M_{k-1} + b M_k + c M_{k+1} = r,
//   a = t_k - t_{k-1}, c = t_{k+1} - t_k, b = 2 (a + c),
//   r = 6 ((y_{k+1} - y_k) / c - (y_k - y_{k-1}) / a).
// Forward elimination leaves row k as M_k + c'_k M_{k+1} = d'_k.  In
// homogeneous form (c'_k = P_k / Q_k, d'_k = D_k / Q_k) one row is the
// linear map
//   Q' = b Q - a P,  P' = c Q,  D' = r Q - a D,
// and a end row the map (Q, 0, 0), which forgets the system before it.  The
// maps of consecutive rows compose associatively, so the forward
// elimination of all rows is a block-wide scan of 3x3 maps of the shape
// [[A, 0], [v^T, s]] (A 2x2), applied to (1, 0, 0).  Back-substitution,
// M_k = d'_k - c'_k M_{k+1}, is a scan of affine maps run from the end.  The
// result is the exact tridiagonal solution (no truncated coupling); scaling
// the homogeneous quantities by powers of two changes no ratio, so they are
// renormalized exactly wherever they could leave the exponent range.

// The equation of row k (0 <= k < n1 + n2; the systems are knots [0, n1)
// and [n1, n1 + n2)): coefficients a, b, c, r, and for segment k (not on a
// system's last knot) its slope, length g and 1/g.
__device__ __forceinline__ void spline_row(const Knots ks, int n1, int n2, int k, double& a,
                                           double& b, double& c, double& r, double& slope,
                                           double& g, double& ig, double& yk) {
  const bool first = k == 0 || k == n1;
  const bool last = k == n1 - 1 || k == n1 + n2 - 1;
  const int t0 = ks.t[k];
  const double y0 = ks.y[k];
  yk = y0;
  double s0 = 0.0, s1 = 0.0, g0 = 0.0, g1 = 0.0, i1 = 0.0;
  if (!last) {
    const int tp = ks.t[k + 1];
    g1 = (double)(tp - t0);
    i1 = recip(g1);
    s1 = (ks.y[k + 1] - y0) * i1;
  }
  if (!first) {
    const int tm = ks.t[k - 1];
    g0 = (double)(t0 - tm);
    s0 = (y0 - ks.y[k - 1]) * recip(g0);
  }
  slope = s1;
  g = g1;
  ig = i1;
  if (first || last) {
    a = 0.0; b = 1.0; c = 0.0; r = 0.0;
  } else {
    a = g0; c = g1; b = 2.0 * (g0 + g1); r = 6.0 * (s1 - s0);
  }
}

// LDS head layout: block-scan ints and the SD sums (256 B), the forward
// wave aggregates (7 doubles per wave), the backward ones (2 per wave).
constexpr int kWaggBytes = 256;
constexpr int kScanFwdBytes = kFwdStride * 16 * (int)sizeof(double);
constexpr int kScanBwdBytes = 2 * 16 * (int)sizeof(double);
constexpr int kAggBytes = kWaggBytes + kScanFwdBytes + kScanBwdBytes;
// Bytes of the detection's published block ends for NT threads.
__host__ __device__ constexpr int pub_bytes(int NT) {
  return (NT * (2 * (int)sizeof(double) + (int)sizeof(int)) + 15) & ~15;
}

// Second derivatives m and segment coefficients q1, q3 of the knot systems
// [0, n1) and [n1, n1 + n2) (n2 = 0: one system).  On [t_k, t_{k+1}), with
// B = k' - t_k and g = t_{k+1} - t_k, the natural spline is
//   y_k + b_k B + (m_k / 2) B^2 + ((m_{k+1} - m_k) / (6 g)) B^3,
//   b_k = (y_{k+1} - y_k) / g - g (2 m_k + m_{k+1}) / 6;
// the walker evaluates half of it (the envelope mean is the sum of the two
// halves), so q1 = b_k / 2 and q3 = (m_{k+1} - m_k) / (12 g) are stored.
// Up to one row per thread of the workgroup, the rows go one per thread
// over as many waves as they need, their data kept in registers;
// otherwise in blocks of R rows per thread over all waves, the forward
// factors c', d' parked in m and q1 of the thread's own rows.  Contains two
// barriers and ends with a third.
template <int NT>
__device__ __forceinline__ void solve_envelopes(const Knots ks, int n1, int n2, int tid,
                                                double* fwd_lds, double* bwd_lds) {
  constexpr int NW = NT / kWave;
  static_assert(NW <= 16, "wave aggregates sized for 16 waves");
  const int rows = n1 + n2;
  const int lane = tid & (kWave - 1), wid = tid / kWave;
  if (rows <= NT) {
    const int wact = (rows + kWave - 1) / kWave;
    const bool wave_active = wid < wact;
    const int k = tid;
    const bool has = k < rows;
    const bool last = k == n1 - 1 || k == n1 + n2 - 1;
    double a = 0.0, b = 1.0, c = 0.0, r = 0.0, sl = 0.0, g = 0.0, ig = 0.0, yk = 0.0;
    FwdMap G = fwd_identity();
    if (has) {
      spline_row(ks, n1, n2, k, a, b, c, r, sl, g, ig, yk);
      G = {b, -a, c, 0.0, r, 0.0, -a};
      fwd_normalize(G);
    }
    if (wave_active) {
      G = fwd_wave_scan(G);
      if (lane == kWave - 1) {
        double* o = fwd_lds + kFwdStride * wid;
        o[0] = G.a00; o[1] = G.a01; o[2] = G.a10; o[3] = G.a11;
        o[4] = G.v0; o[5] = G.v1; o[6] = G.s;
      }
    }
    __syncthreads();
    double cp = 0.0, dp = 0.0, al = 0.0, be = 1.0;
    if (wave_active) {
      double Q, P, D;
      fwd_enter(fwd_lds, wid, Q, P, D);
      fwd_apply(fwd_dpp<kDppWaveShr1, 0xf>(G), Q, P, D);  // (lane 0: the identity)
      if (has) {
        const double q = fma(b, Q, -a * P);
        D = fma(r, Q, -a * D);
        P = c * Q;
        const double iq = recip(q);
        cp = P * iq;
        dp = D * iq;
        al = dp;
        be = -cp;
      }
      bwd_wave_scan(al, be, lane);
      if (lane == 0) {
        bwd_lds[2 * wid] = al;
        bwd_lds[2 * wid + 1] = be;
      }
    }
    __syncthreads();
    if (wave_active) {
      double Mn = bwd_after(bwd_lds, wid, wact);
      // (lane 63: the identity x -> 0 + 1 x)
      Mn = fma(dpp_move<kDppWaveShl1, 0xf, true>(be), Mn, dpp_move<kDppWaveShl1, 0xf>(al));
      if (has) {
        const double Mk = fma(-cp, Mn, dp);
        if (!last) {
          ks.q1[k] = 0.5 * (sl - g * fma(2.0, Mk, Mn) * (1.0 / 6.0));
          ks.q3[k] = (Mn - Mk) * ig * (1.0 / 12.0);
        }
        ks.m[k] = 0.25 * Mk;
        ks.y[k] = 0.5 * yk;
      }
    }
    __syncthreads();
    return;
  }

  // more rows than threads: blocks of R rows per thread over all waves
  // (R a multiple of 4 is raised by one: row blocks whose starts lie a
  // multiple of 8 doubles apart would share LDS banks 4 ways or more)
  int R = (rows + NT - 1) / NT;
  R += (R & 3) == 0 ? 1 : 0;
  const int k0 = tid * R, k1 = min(rows, k0 + R);
  FwdMap G = fwd_identity();
  for (int k = k0; k < k1; ++k) {
    double a, b, c, r, sl, g, ig, yk;
    spline_row(ks, n1, n2, k, a, b, c, r, sl, g, ig, yk);
    G = fwd_row_after(a, b, c, r, G);
    if (((k - k0) & 3) == 3) fwd_normalize(G);
  }
  fwd_normalize(G);
  G = fwd_wave_scan(G);
  if (lane == kWave - 1) {
    double* o = fwd_lds + kFwdStride * wid;
    o[0] = G.a00; o[1] = G.a01; o[2] = G.a10; o[3] = G.a11;
    o[4] = G.v0; o[5] = G.v1; o[6] = G.s;
  }
  __syncthreads();
  {
    double Q, P, D;
    fwd_enter(fwd_lds, wid, Q, P, D);
    fwd_apply(fwd_dpp<kDppWaveShr1, 0xf>(G), Q, P, D);  // (lane 0: the identity)
    vec_normalize(Q, P, D);
    // each row's c' (into m) and d' (into q1): rows of this thread only
    for (int k = k0; k < k1; ++k) {
      double a, b, c, r, sl, g, ig, yk;
      spline_row(ks, n1, n2, k, a, b, c, r, sl, g, ig, yk);
      const double q = fma(b, Q, -a * P);
      D = fma(r, Q, -a * D);
      P = c * Q;
      Q = q;
      vec_normalize(Q, P, D);
      const double iq = recip(Q);
      ks.m[k] = P * iq;
      ks.q1[k] = D * iq;
    }
  }
  // back-substitution maps composed from the thread's last row down
  double al = 0.0, be = 1.0;
  for (int k = k1 - 1; k >= k0; --k) {
    const double cp = ks.m[k], dp = ks.q1[k];
    al = fma(-cp, al, dp);
    be = -cp * be;
  }
  bwd_wave_scan(al, be, lane);
  if (lane == 0) {
    bwd_lds[2 * wid] = al;
    bwd_lds[2 * wid + 1] = be;
  }
  __syncthreads();
  {
    double Mn = bwd_after(bwd_lds, wid, NW);
    // (lane 63: the identity x -> 0 + 1 x)
    Mn = fma(dpp_move<kDppWaveShl1, 0xf, true>(be), Mn, dpp_move<kDppWaveShl1, 0xf>(al));
    for (int k = k1 - 1; k >= k0; --k) {
      const double cp = ks.m[k], dp = ks.q1[k];
      const double Mk = fma(-cp, Mn, dp);
      const bool last = k == n1 - 1 || k == n1 + n2 - 1;
      if (!last) {
        const double g = (double)((int)ks.t[k + 1] - (int)ks.t[k]);
        const double ig = recip(g);
        const double bk = (ks.y[k + 1] - ks.y[k]) * ig - g * fma(2.0, Mk, Mn) * (1.0 / 6.0);
        ks.q1[k] = 0.5 * bk;
        ks.q3[k] = (Mn - Mk) * ig * (1.0 / 12.0);
      }
      ks.m[k] = 0.25 * Mk;
      Mn = Mk;
    }
  }
  __syncthreads();  // the values of the neighbours' rows have been read
  for (int k = k0; k < k1; ++k) ks.y[k] = 0.5 * ks.y[k];
  __syncthreads();
}

// Walker over the segments of one envelope: the current segment j =
// [t_j, t1), its halved power-form coefficients and the local abscissa
// B = k - t_j.
struct Walk {
  int j, t1;
  double B, q0, q1, q2, q3;
};

__device__ __forceinline__ void walk_load(Walk& w, const Knots& ks, int j) {
  w.j = j;
  w.t1 = ks.t[j + 1];
  w.q0 = ks.y[j];
  w.q1 = ks.q1[j];
  w.q2 = ks.m[j];
  w.q3 = ks.q3[j];
}

// Position at the segment holding sample k, starting from segment j (whose
// left knot lies at or before k; the last knot lies beyond the signal).
__device__ __forceinline__ void walk_init(Walk& w, const Knots& ks, int j, int k) {
  int t0 = ks.t[j];
  walk_load(w, ks, j);
  while (w.t1 <= k) {
    t0 = w.t1;
    walk_load(w, ks, w.j + 1);
  }
  w.B = (double)(k - t0);
}

// Half the envelope at sample k, the walker standing at k (knots are
// distinct integers, so one step from k-1 crosses at most one of them, and
// the new segment starts where the old one ends).
__device__ __forceinline__ double walk_at(Walk& w, const Knots& ks, int k) {
  if (w.t1 <= k) {
    w.B = (double)(k - w.t1);
    walk_load(w, ks, w.j + 1);
  }
  return fma(fma(fma(w.q3, w.B, w.q2), w.B, w.q1), w.B, w.q0);
}

// h[c] for a lane-dependent c, by selects.  Each element passes through an
// empty asm so that the selects cannot be folded back into an indexed load,
// which would move the whole array out of registers into scratch memory.
template <int C>
__device__ __forceinline__ double pick(const double (&h)[C], int c) {
  double y = h[0];
  asm volatile("" : "+v"(y));
#pragma unroll
  for (int j = 1; j < C; ++j) {
    double v = h[j];
    asm volatile("" : "+v"(v));
    y = (c == j) ? v : y;
  }
  return y;
}

// The mirrored end knots of one kind (Sec. 2.1 Step 2 with the mirror
// boundary) held by this thread: its knots of that kind (bits) have ranks
// e.. among n, and ranks 0, 1, n-2, n-1 are mirrored about samples 0 and L-1.
template <int C>
__device__ __forceinline__ void emit_mirrors(const double (&h)[C], unsigned bits, unsigned NE,
                                             int carry, int base, int L, int e, int n,
                                             const Knots ks) {
  const int cnt = __popc(bits);
  if (cnt == 0 || (e >= 2 && e + cnt <= n - 2)) return;
  const int Pp = n < 2 ? n : 2;
  const int hi = 2 * (L - 1);
  int g = e;
  while (bits) {
    const int c = __ffs(bits) - 1;
    bits &= bits - 1u;
    if (g < 2 || g >= n - 2) {
      const int mid = run_mid(NE, carry, base, c);
      const double y = pick(h, c);
      if (g == 0) { ks.t[Pp - 1] = (int16_t)(-mid); ks.y[Pp - 1] = y; }
      if (g == 1 && Pp == 2) { ks.t[0] = (int16_t)(-mid); ks.y[0] = y; }
      if (g == n - 1) { ks.t[Pp + n] = (int16_t)(hi - mid); ks.y[Pp + n] = y; }
      if (g == n - 2 && Pp == 2) { ks.t[Pp + n + 1] = (int16_t)(hi - mid); ks.y[Pp + n + 1] = y; }
    }
    ++g;
  }
}

// Both kinds of knots, each thread walking its own extrema: maxima go to ku
// (first rank emax of nmax), minima to kl (first rank emin of nmin).
template <int C>
__device__ __forceinline__ void rd_emit_both(const double (&h)[C], unsigned maxbits,
                                             unsigned minbits, unsigned NE, int carry, int base,
                                             int L, int emax, int nmax, int emin, int nmin,
                                             const Knots ku, const Knots kl) {
  const int Pu = nmax < 2 ? nmax : 2, Pl = nmin < 2 ? nmin : 2;
  unsigned any = maxbits | minbits;
  while (any) {
    const int c = __ffs(any) - 1;
    any &= any - 1u;
    const bool up = (maxbits >> c) & 1u;
    const unsigned below = (1u << c) - 1u;
    const int g = up ? Pu + emax + __popc(maxbits & below) : Pl + emin + __popc(minbits & below);
    const int mid = run_mid(NE, carry, base, c);
    const double y = pick(h, c);
    int16_t* t = up ? ku.t : kl.t;
    double* yy = up ? ku.y : kl.y;
    t[g] = (int16_t)mid;
    yy[g] = y;
  }
  emit_mirrors(h, maxbits, NE, carry, base, L, emax, nmax, ku);
  emit_mirrors(h, minbits, NE, carry, base, L, emin, nmin, kl);
}

// Second derivatives and segment coefficients of the emitted knot systems
// (n1 knots at offset 0, n2 at offset n1); the knots must be complete (a
// barrier after emission).  Ends with a barrier.
template <int NT>
__device__ __forceinline__ void finish_envelopes(const Knots ks, int nk1, int nk2, int tid) {
  extern __shared__ __align__(16) unsigned char smem[];
  solve_envelopes<NT>(ks, nk1, nk2, tid, reinterpret_cast<double*>(smem + kWaggBytes),
                      reinterpret_cast<double*>(smem + kWaggBytes + kScanFwdBytes));
}

// One envelope (single-envelope mode): emitted, solved, coefficients formed.
template <int NT, int C>
__device__ __forceinline__ void build_envelope(const double (&h)[C], unsigned bits, unsigned NE,
                                               int carry, int base, int L, int first, int n,
                                               const Knots ks, int nk, int tid) {
  rd_emit<C>(h, bits, NE, carry, base, L, first, n, ks);
  __syncthreads();
  finish_envelopes<NT>(ks, nk, 0, tid);
}

// One sift with both envelopes in one knot store: build, then evaluate both
// walkers per sample and subtract the mean (Sec. 2.1 Steps 2-4).  Adds the
// thread's sums of m^2 and of the candidate's h^2 before the sift to num, den.
template <int NT, int C>
__device__ __forceinline__ void sift_both(double (&h)[C], unsigned maxbits, unsigned minbits,
                                          unsigned NE, int carry, int base, int nv, int L,
                                          int emax, int nmax, int pmax, int emin, int nmin,
                                          int pmin, const Knots ks, int nkmax, int nkmin,
                                          int tid, double& num, double& den) {
  rd_emit_both<C>(h, maxbits, minbits, NE, carry, base, L, emax, nmax, emin, nmin, ks,
                  knots_from(ks, nkmax));
  __syncthreads();
  finish_envelopes<NT>(ks, nkmax, nkmin, tid);
  if (nv > 0) {
    const Knots kl = knots_from(ks, nkmax);
    Walk wu, wl;
    walk_init(wu, ks, pmax + emax - 1, base);
    walk_init(wl, kl, pmin + emin - 1, base);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if (c < nv) {
        const int k = base + c;
        const double up = walk_at(wu, ks, k);
        const double lo = walk_at(wl, kl, k);
        const double m = up + lo;
        num = fma(m, m, num);
        den = fma(h[c], h[c], den);
        h[c] = h[c] - m;
        wu.B += 1.0;
        wl.B += 1.0;
      }
    }
  }
}

// Hides a value's origin from the optimizer (no instruction is emitted).
__device__ __forceinline__ void opaque(int& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(unsigned& v) { asm volatile("" : "+v"(v)); }

// Position in the staging window of chunk sample j (blocks of C samples,
// each followed by one spare double).
template <int C>
__device__ __forceinline__ int stage_at(int j) { return j + j / C; }

// Samples of the chunk [c0, c1) of the signal that thread-owned slot c maps to.
__device__ __forceinline__ bool in_chunk(int k, int c0, int c1) { return k >= c0 && k < c1; }

// k / R and k % R for 0 <= k < 2^24 and R >= 1 from a float reciprocal,
// corrected by one step either way.
__device__ __forceinline__ void div_small(int k, int R, float invR, int& q, int& rem) {
  q = (int)((float)k * invR);
  rem = k - q * R;
  if (rem < 0) { --q; rem += R; }
  else if (rem >= R) { ++q; rem -= R; }
}

// ---------------------------------------------------------------------------
// Resident Serial-EMD kernel: one workgroup per work item
// ---------------------------------------------------------------------------

// LDS: the head (wave totals and the spline scans' wave aggregates), the
// published block ends of the extremum detection (20 B per thread), then one
// area (area_bytes) used in turn as
//   - a staging window of the signal (a multiple of NT doubles) at load and
//     IMF ends, so global reads and writes stay coalesced;
//   - the knot store (34 B per knot).
// Detection writes only its own region, so a sift starts while slower waves
// still evaluate the previous sift's envelopes from the knot store.
// A sift keeps both envelopes' knots in LDS when they fit together (one
// solve, one fused evaluation, mean and update); else one envelope at a time
// when each fits (the upper envelope parked in global memory); else both in
// the item's global knot store.
template <int NT, int C, bool TRACE = false>
__global__ void __launch_bounds__(NT) resident_emd_kernel(const WorkItem* __restrict__ items,
                                                          int K, int S, int area_bytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = NT / kWave;
  static_assert(2 * NW * sizeof(double) <= kWaggBytes, "wave sums exceed the LDS head");
  const int tid0 = threadIdx.x;
  const WorkItem w = items[blockIdx.x];
  // the resident path holds at most kResidentMaxL samples: 32-bit indices
  const int L = w.L;
  const int M = (int)w.M, MN = (int)(w.M * w.N), R = (int)(w.M + w.D);
  const int D = w.D;
  const float invR = 1.0f / (float)R;

  int* wagg = reinterpret_cast<int*>(smem);
  double* pub_first = reinterpret_cast<double*>(smem + kAggBytes);
  double* pub_last = pub_first + NT;
  int* pub_key = reinterpret_cast<int*>(pub_last + NT);
  unsigned char* area = smem + kAggBytes + pub_bytes(NT);
  const int capk = area_bytes / kKnotBytes;  // knots the LDS store can take
  // Staging window for loads and IMF ends: the samples of whole thread
  // blocks, each block followed by one spare double, so that the blocked
  // accesses (stride C + 1 doubles, C even) fall on distinct LDS banks.
  const int scap = (area_bytes / (int)sizeof(double)) / (C + 1) * C;
  double* stage = reinterpret_cast<double*>(area);
  const Knots lk = knots_in(area, capk);
  const Knots gk = knots_in(reinterpret_cast<unsigned char*>(w.u), resident_gknot_cap(L));

  const int base0 = tid0 * C;
  const int nv0 = max(0, min(C, L - base0));

  // Load: serialize (Sec. 3.2), add the realization's noise (Sec. 2.2 Step 1)
  double h[C];
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = 0.0;
  int bad = 0;
  for (int c0 = 0; c0 < L; c0 += scap) {
    const int c1 = min(L, c0 + scap);
    __syncthreads();
    for (int k0 = c0 + tid0; k0 < c1; k0 += 4 * NT) {
      // four elements per pass, formed before any of their stores (an input
      // read cannot move above a store to r, which might alias the input)
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u * NT;
        v[u] = 0.0;
        if (k < c1) {
          int i, m;
          div_small(k, R, invR, i, m);
          v[u] = (w.flags & kNoSignal) ? 0.0 : serial_at(w.X, M, D, i, m);
          if (w.flags & (kAddNoise | kAddBuffer)) {
            const double b = (w.flags & kScaleOnDevice) ? *w.scale : w.beta;
            const double e = (w.flags & kAddNoise) ? noise_at(w.key, k) : w.addend[k];
            v[u] = __dadd_rn(v[u], __dmul_rn(b, e));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u * NT;
        if (k < c1) {
          bad |= !isfinite(v[u]);
          stage[stage_at<C>(k - c0)] = v[u];
          w.r[k] = v[u];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (c < nv0 && in_chunk(base0 + c, c0, c1)) h[c] = stage[stage_at<C>(base0 - c0) + c];
  }
  const int64_t SS = w.slot_stride;
  // extremum-decision trace: entries used (the same in every thread) and
  // whether every record so far fitted
  int tr_used = 4, tr_ok = 1;
  if (__syncthreads_or(bad)) {
    for (int q = 0; q <= K; ++q)
      for (int o = tid0; o < MN; o += NT) w.out[q * SS + o] = 0.0;
    if (tid0 == 0 && w.n_imfs) *w.n_imfs = -5;
    if constexpr (TRACE) {
      if (tid0 == 0) {
        w.trace[0] = tr_used;
        w.trace[1] = tr_ok;
      }
    }
    return;
  }

  int nimf = 0;
  int64_t n_sifts = 0, n_knots = 0;
  while (nimf < K) {
    bool stop = false;
    for (int s = 0; s < S; ++s) {
      // Values derived from the thread's position are recomputed every sift
      // rather than hoisted out of the loop and held in registers throughout.
      int tid = tid0, base = base0, nv = nv0;
      opaque(tid);
      opaque(base);
      opaque(nv);
      unsigned Rm, Fm, maxbits, minbits;
      int carry;
      rd_detect<NT, C>(h, base, nv, L, tid, pub_first, pub_last, pub_key, Rm, Fm, carry,
                       maxbits, minbits);
      // The masks are kept as masks: otherwise their popcounts get rebuilt
      // from the individual comparison bits, all of which then stay live.
      opaque(maxbits);
      opaque(minbits);
      opaque(Rm);
      opaque(Fm);
      int tot;
      int excl = block_excl_sum<NW>((__popc(maxbits) << 16) | __popc(minbits), wagg,
                                    tid & (kWave - 1), tid / kWave, tot);
      // (summed now: otherwise the wave totals stay live, one register each,
      // until the ranks are used)
      opaque(excl);
      opaque(tot);
      const int nmax = tot >> 16, nmin = tot & 0xffff;
      if constexpr (TRACE) {
        // record (imf, sift, counts, positions) of this detection
        const int need = 4 + nmax + nmin;
        if (tr_ok && tr_used + need <= w.trace_cap) {
          int32_t* rec = w.trace + tr_used;
          if (tid == 0) {
            rec[0] = nimf;
            rec[1] = s;
            rec[2] = nmax;
            rec[3] = nmin;
          }
          const unsigned ne = Rm | Fm;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const unsigned below = (1u << c) - 1u;
            if ((maxbits >> c) & 1u)
              rec[4 + (excl >> 16) + __popc(maxbits & below)] = run_mid(ne, carry, base, c);
            if ((minbits >> c) & 1u)
              rec[4 + nmax + (excl & 0xffff) + __popc(minbits & below)] =
                  run_mid(ne, carry, base, c);
          }
          tr_used += need;
        } else {
          tr_ok = 0;
        }
      }
      if (!(nmax >= 1 && nmin >= 1 && nmax + nmin >= 3)) {
        stop = (s == 0);  // the residue itself is not siftable: decomposition ends
        break;
      }
      const unsigned NE = Rm | Fm;
      const int emax = excl >> 16, emin = excl & 0xffff;
      const int pmax = nmax < 2 ? nmax : 2, pmin = nmin < 2 ? nmin : 2;
      const int nkmax = nmax + 2 * pmax, nkmin = nmin + 2 * pmin;
      ++n_sifts;
      n_knots += nkmax + nkmin;
      const bool both_lds = nkmax + nkmin <= capk;
      const bool single = !both_lds && nkmax <= capk && nkmin <= capk;
      double num = 0.0, den = 0.0;
      if (both_lds) {
        // both envelopes at once in LDS: one solve, fused evaluation and update
        sift_both<NT, C>(h, maxbits, minbits, NE, carry, base, nv, L, emax, nmax, pmax, emin,
                         nmin, pmin, lk, nkmax, nkmin, tid, num, den);
      } else if (single) {
        // one envelope at a time in LDS, the upper one parked in global memory
        build_envelope<NT, C>(h, maxbits, NE, carry, base, L, emax, nmax, lk, nkmax, tid);
        if (nv > 0) {
          Walk wu;
          walk_init(wu, lk, pmax + emax - 1, base);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if (c < nv) {
              w.u[base + c] = walk_at(wu, lk, base + c);
              wu.B += 1.0;
            }
          }
        }
        __syncthreads();
        build_envelope<NT, C>(h, minbits, NE, carry, base, L, emin, nmin, lk, nkmin, tid);
        if (nv > 0) {
          Walk wl;
          walk_init(wl, lk, pmin + emin - 1, base);
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if (c < nv) {
              const double lo = walk_at(wl, lk, base + c);
              const double m = w.u[base + c] + lo;
              num = fma(m, m, num);
              den = fma(h[c], h[c], den);
              h[c] = h[c] - m;
              wl.B += 1.0;
            }
          }
        }
      } else {
        // both envelopes in the item's global knot store
        sift_both<NT, C>(h, maxbits, minbits, NE, carry, base, nv, L, emax, nmax, pmax, emin,
                         nmin, pmin, gk, nkmax, nkmin, tid, num, den);
      }
      // SD criterion: the IMF ends after a sift whose mean is small against
      // the candidate it was removed from (every thread sees the same sums)
      if (w.sd > 0.0) {
        double tnum, tden;
        block_sum2<NW>(num, den, reinterpret_cast<double*>(wagg), tid & (kWave - 1),
                       tid / kWave, tnum, tden);
        if (tnum < w.sd * tden) break;
      }
    }
    if (stop) break;
    // IMF nimf = h (deserialized store, Sec. 3.3); residue r <- r - h; h <- r
    double* slot = w.out + (int64_t)nimf * SS;
    int tid = tid0, base = base0, nv = nv0;
    opaque(tid);
    opaque(base);
    opaque(nv);
    for (int c0 = 0; c0 < L; c0 += scap) {
      const int c1 = min(L, c0 + scap);
      __syncthreads();
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (c < nv && in_chunk(base + c, c0, c1)) stage[stage_at<C>(base - c0) + c] = h[c];
      __syncthreads();
      for (int k0 = c0 + tid; k0 < c1; k0 += 4 * NT) {
        // four elements per pass, their residue loads issued together
        double rk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + u * NT;
          rk[u] = k < c1 ? w.r[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + u * NT;
          if (k < c1) {
            const int si = stage_at<C>(k - c0);
            const double hk = stage[si];
            const double nr = rk[u] - hk;
            w.r[k] = nr;
            stage[si] = nr;
            int i, m;
            div_small(k, R, invR, i, m);
            if (m < M) slot[i * M + m] = hk;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (c < nv && in_chunk(base + c, c0, c1)) h[c] = stage[stage_at<C>(base - c0) + c];
    }
    ++nimf;
  }
  // residue into slot K (every r[k] was last written by this same thread),
  // unused IMF slots zero (Sec. 4.3 zero fill)
  double* rslot = w.out + (int64_t)K * SS;
  for (int k0 = tid0; k0 < L; k0 += 4 * NT) {
    double rk[4];  // (loaded together, before the stores)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * NT;
      rk[u] = k < L ? w.r[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + u * NT;
      if (k < L) {
        int i, m;
        div_small(k, R, invR, i, m);
        if (m < M) rslot[i * M + m] = rk[u];
      }
    }
  }
  for (int q = nimf; q < K; ++q)
    for (int o = tid0; o < MN; o += NT) w.out[q * SS + o] = 0.0;
  if (tid0 == 0 && w.n_imfs) *w.n_imfs = nimf;
  if constexpr (TRACE) {
    if (tid0 == 0) {
      w.trace[0] = tr_used;
      w.trace[1] = tr_ok;
    }
  }
  if (tid0 == 0 && w.stats) {
    w.stats[0] = n_sifts;
    w.stats[1] = n_knots;
    w.stats[2] = n_sifts * (int64_t)L;
  }
}

// Extrema of one signal by the resident kernel's detection and ranking:
// sorted maximum and minimum indices, and their counts.
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
  unsigned R, F, maxbits, minbits;
  int carry;
  rd_detect<NT, C>(h, base, nv, L, tid, pub_first, pub_last, pub_key, R, F, carry, maxbits,
                   minbits);
  int tot;
  const int excl = block_excl_sum<NW>((__popc(maxbits) << 16) | __popc(minbits), wagg, lane,
                                      wid, tot);
  const unsigned NE = R | F;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    if ((maxbits >> c) & 1u)
      imax[(excl >> 16) + __popc(maxbits & ((1u << c) - 1u))] = run_mid(NE, carry, base, c);
    if ((minbits >> c) & 1u)
      imin[(excl & 0xffff) + __popc(minbits & ((1u << c) - 1u))] = run_mid(NE, carry, base, c);
  }
  if (tid == 0) {
    counts[0] = tot >> 16;
    counts[1] = tot & 0xffff;
  }
}

// ---------------------------------------------------------------------------
// Streaming helper kernels
// ---------------------------------------------------------------------------

// dst[0] = w: the descriptor of a single-signal launch, handed over as a
// kernel argument so that no host staging buffer is involved.
__global__ void put_work_kernel(WorkItem w, WorkItem* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = w;
}

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

// Tuning input: n signals of L samples, signal i at x + i*L: two sinusoids
// and white noise, x[k] = sin(2 pi k / 37.3) + 0.6 sin(2 pi k / 9.7 + i)
// + 0.25 w_i[k].
__global__ void synth_kernel(double* __restrict__ x, int64_t L, int n, uint64_t seed) {
  const int64_t total = L * n;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / L, k = q - i * L;
    const double t = (double)k;
    x[q] = sin(2.0 * M_PI * t / 37.3) + 0.6 * sin(2.0 * M_PI * t / 9.7 + (double)i) +
           0.25 * noise_at(noise_key(seed, (uint64_t)i, 0), k);
  }
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

// dst[j] = sum over m of src[3m + j], j < 3: work statistics of NR realizations.
__global__ void sum_stats_kernel(const int64_t* __restrict__ src, int NR,
                                 int64_t* __restrict__ dst) {
  const int j = threadIdx.x;
  if (blockIdx.x == 0 && j < 3) {
    int64_t acc = 0;
    for (int m = 0; m < NR; ++m) acc += src[3 * m + j];
    dst[j] = acc;
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

// Compute units of the current device (queried once).
int device_cus() {
  static const int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v < 1)
      v = 256;
    return v;
  }();
  return cus;
}

template <int NT, int C, bool TRACE = false>
hipError_t launch_resident_cls(const WorkItem* d_items, int n, int maxL, int K, int S,
                               hipStream_t stream) {
  auto kern = resident_emd_kernel<NT, C, TRACE>;
  static const hipFuncAttributes attr = [&] {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kern)) != hipSuccess) {
      a.sharedSizeBytes = 1024;
      a.numRegs = 256;
    }
    return a;
  }();
  // Workgroups a CU can hold by registers (512 VGPRs per SIMD lane, four
  // SIMDs), and how many it will be given: the LDS is shared out among them.
  constexpr size_t kLdsPerCU = 160 * 1024;
  const int regs = std::max(8, (attr.numRegs + 7) / 8 * 8);
  const int waves_simd = std::max(1, std::min(8, 512 / regs));
  int wg_cu = std::max(1, waves_simd * 4 / (NT / kWave));
  wg_cu = std::min(wg_cu, std::max(1, (n + device_cus() - 1) / device_cus()));
  const size_t per_wg = (kLdsPerCU / (size_t)wg_cu) & ~size_t(511);
  const size_t limit = std::min(per_wg, kLdsPerCU) - (size_t)attr.sharedSizeBytes;
  const size_t head = kAggBytes + pub_bytes(NT);
  const size_t area = resident_area_bytes(maxL, NT, limit - head);
  const size_t lds = head + area;
  if (lds > kLdsPerCU - (size_t)attr.sharedSizeBytes) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n), dim3(NT), lds, stream, d_items, K, S, (int)area);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CEEMDAN stages (Sec. 2.2): per-item bookkeeping between the ensembles of
// first-mode extractions, one workgroup per item
// ---------------------------------------------------------------------------

constexpr int kCT = 256;  // threads of the CEEMDAN kernels

// Can v[0..L) be sifted (>= 1 maximum, >= 1 minimum, >= 3 extrema)?  The
// extrema are counted as changes of direction between consecutive steps
// (pairs of unequal neighbouring samples): a rise then a fall brackets one
// maximum, strict or an equal-valued run, a fall then a rise one minimum,
// and a run touching an end has no step on that side.  Each thread counts
// its own stretch of steps; thread 0 joins the stretches in order.
__device__ bool block_siftable(const double* v, int64_t L, int* sc) {
  __shared__ int flag;
  const int tid = threadIdx.x;
  if (L < 3) return false;
  const int64_t pairs = L - 1;
  const int64_t chunk = (pairs + kCT - 1) / kCT;
  const int64_t a = min((int64_t)tid * chunk, pairs), b = min(a + chunk, pairs);
  int first = 0, last = 0, nmax = 0, nmin = 0;
  for (int64_t k = a; k < b; ++k) {
    const double d0 = v[k], d1 = v[k + 1];
    const int d = d1 > d0 ? 1 : (d1 < d0 ? -1 : 0);
    if (d != 0) {
      if (last != 0 && last != d) {
        if (last > 0) ++nmax;
        else ++nmin;
      }
      if (first == 0) first = d;
      last = d;
    }
  }
  sc[4 * tid] = first;
  sc[4 * tid + 1] = last;
  sc[4 * tid + 2] = nmax;
  sc[4 * tid + 3] = nmin;
  __syncthreads();
  if (tid == 0) {
    int prev = 0, tmax = 0, tmin = 0;
    for (int t = 0; t < kCT; ++t) {
      const int f = sc[4 * t];
      if (f == 0) continue;
      if (prev != 0 && prev != f) {
        if (prev > 0) ++tmax;
        else ++tmin;
      }
      tmax += sc[4 * t + 2];
      tmin += sc[4 * t + 3];
      prev = sc[4 * t + 1];
    }
    flag = (tmax >= 1 && tmin >= 1 && tmax + tmin >= 3) ? 1 : 0;
  }
  __syncthreads();
  const bool ok = flag != 0;
  __syncthreads();
  return ok;
}

// Sum of v[0..L) (f = 0) or of (v - mean)^2 (f = 1): each thread sums its
// stretch in order, thread 0 the stretches in order.
__device__ double block_sum_dev(const double* v, int64_t L, double mean, int f, double* sd) {
  __shared__ double total;
  const int tid = threadIdx.x;
  const int64_t chunk = (L + kCT - 1) / kCT;
  const int64_t a = min((int64_t)tid * chunk, L), b = min(a + chunk, L);
  double acc = 0.0;
  for (int64_t k = a; k < b; ++k) {
    const double x = v[k];
    if (f == 0) {
      acc = acc + x;
    } else {
      const double d = x - mean;
      acc = acc + d * d;
    }
  }
  sd[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < kCT; ++i) t = t + sd[i];
    total = t;
  }
  __syncthreads();
  const double r = total;
  __syncthreads();
  return r;
}

// The residue's siftability and the next stage's noise amplitude
// eps * std(r) (population standard deviation).
__device__ void ceemdan_assess(const CeemdanJob& J, int* sc, double* sd) {
  const bool ok = block_siftable(J.r, J.L, sc);
  const double mean = block_sum_dev(J.r, J.L, 0.0, 0, sd) / (double)J.L;
  const double q = block_sum_dev(J.r, J.L, mean, 1, sd);
  if (threadIdx.x == 0) {
    J.st->alive = ok ? 1 : 0;
    J.st->scale = J.eps * sqrt(q / (double)J.L);
  }
}

__global__ void __launch_bounds__(kCT) ceemdan_prep_kernel(const CeemdanJob* __restrict__ jobs,
                                                           int K) {
  __shared__ int sc[4 * kCT];
  __shared__ double sd[kCT];
  const CeemdanJob J = jobs[blockIdx.x];
  const int64_t KL = (int64_t)K * J.L;
  for (int64_t i = threadIdx.x; i < KL; i += kCT) J.modes[i] = 0.0;
  int bad = 0;
  for (int64_t k = threadIdx.x; k < J.L; k += kCT) bad |= !isfinite(J.r[k]);
  bad = __syncthreads_or(bad);
  if (bad) {
    if (threadIdx.x == 0) {
      J.st->alive = 0;
      J.st->scale = 0.0;
      J.st->n = -5;
    }
    return;
  }
  if (threadIdx.x == 0) J.st->n = 0;
  ceemdan_assess(J, sc, sd);
}

// Mode `stage` of item blockIdx.x, samples of tile blockIdx.y: the mean of
// the NR first modes (summed in m order) into the mode slot, r -= mode.
constexpr int kCTile = kCT * 8;
__global__ void __launch_bounds__(kCT) ceemdan_combine_kernel(const CeemdanJob* __restrict__ jobs,
                                                              int stage) {
  const CeemdanJob J = jobs[blockIdx.x];
  if (!J.st->alive) return;
  double* mode = J.modes + (int64_t)(stage - 1) * J.L;
  const int64_t L2 = 2 * J.L;
  const int64_t k0 = (int64_t)blockIdx.y * kCTile;
  const int64_t k1 = min(J.L, k0 + kCTile);
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kCT) {
    double acc = 0.0;
#pragma unroll 8
    for (int m = 0; m < J.NR; ++m) acc = acc + J.stage[m * L2 + k];
    const double c = acc / (double)J.NR;
    mode[k] = c;
    J.r[k] = J.r[k] - c;
  }
}

// After mode `stage`: the mode count, and whether the new residue can still
// be sifted and the next stage's amplitude.
__global__ void __launch_bounds__(kCT) ceemdan_assess_kernel(const CeemdanJob* __restrict__ jobs,
                                                             int stage) {
  __shared__ int sc[4 * kCT];
  __shared__ double sd[kCT];
  const CeemdanJob J = jobs[blockIdx.x];
  const int alive = J.st->alive;
  __syncthreads();  // every thread has read the state before it changes
  if (!alive) return;
  if (threadIdx.x == 0) J.st->n = stage;
  ceemdan_assess(J, sc, sd);
}

__global__ void __launch_bounds__(kCT) ceemdan_finish_kernel(const CeemdanJob* __restrict__ jobs,
                                                             int K) {
  const CeemdanJob J = jobs[blockIdx.x];
  const int q = blockIdx.y;  // output slot 0..K
  const int n = J.st->n;
  const double* src = q < K ? J.modes + (int64_t)q * J.L : J.r;
  const int64_t MN = J.M * J.N, R = J.M + J.D;
  double* dst = J.out + (int64_t)q * J.slot_stride;
  for (int64_t o = threadIdx.x; o < MN; o += kCT) {
    const int64_t i = o / J.M, m = o - i * J.M;
    dst[o] = n < 0 ? 0.0 : src[i * R + m];
  }
  if (q == 0 && threadIdx.x == 0 && J.n_out) *J.n_out = n;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Threads and samples per thread for signals up to maxL samples, for a
// launch of few signals (regime 0: each has a CU to itself) or of at least
// one per CU (regime 1).  Defaults: the shapes the tuner picks on MI355X
// (more threads per signal beat more signals per CU, the sift phases being
// bound by latency, except for short signals in full launches).
ResidentClass resident_class(int maxL, int regime) {
  if (regime == 1 && maxL <= 256 * 4) return {256, 4};
  if (regime == 1 && maxL <= 256 * 8) return {256, 8};
  if (regime == 0 && maxL <= 1024 * 3) return {1024, 4};
  if (maxL <= 512 * 8) return {512, 8};
  if (maxL <= 1024 * 8) return {1024, 8};
  if (maxL <= 1024 * 12) return {1024, 12};
  return {1024, 16};
}

size_t resident_area_bytes(int maxL, int nt, size_t max_area) {
  const size_t stage = (size_t)nt * sizeof(double);
  // both envelopes of any sift (at most L + 6 knots) if the budget allows
  const size_t dual = (size_t)kKnotBytes * ((size_t)maxL + 16);
  size_t area = std::min(dual, max_area);
  area = std::max(area, stage);
  return area & ~size_t(15);
}

// The compiled launch shapes (threads, samples per thread).
static const ResidentClass kClasses[] = {{256, 4},   {256, 8},   {256, 12},  {256, 16},
                                         {512, 8},   {512, 12},  {512, 16},  {1024, 4},
                                         {1024, 8},  {1024, 12}, {1024, 16}};

int resident_classes(ResidentClass* out, int cap) {
  const int n = (int)(sizeof(kClasses) / sizeof(kClasses[0]));
  for (int i = 0; i < n && i < cap; ++i) out[i] = kClasses[i];
  return n;
}

hipError_t launch_resident(const WorkItem* d_items, int n, int maxL, ResidentClass c, int K,
                           int S, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (c.nt * c.c < maxL) return hipErrorInvalidValue;
  switch (c.nt * 100 + c.c) {
    case 25604: return launch_resident_cls<256, 4>(d_items, n, maxL, K, S, stream);
    case 25608: return launch_resident_cls<256, 8>(d_items, n, maxL, K, S, stream);
    case 25612: return launch_resident_cls<256, 12>(d_items, n, maxL, K, S, stream);
    case 25616: return launch_resident_cls<256, 16>(d_items, n, maxL, K, S, stream);
    case 51208: return launch_resident_cls<512, 8>(d_items, n, maxL, K, S, stream);
    case 51212: return launch_resident_cls<512, 12>(d_items, n, maxL, K, S, stream);
    case 51216: return launch_resident_cls<512, 16>(d_items, n, maxL, K, S, stream);
    case 102404: return launch_resident_cls<1024, 4>(d_items, n, maxL, K, S, stream);
    case 102408: return launch_resident_cls<1024, 8>(d_items, n, maxL, K, S, stream);
    case 102412: return launch_resident_cls<1024, 12>(d_items, n, maxL, K, S, stream);
    case 102416: return launch_resident_cls<1024, 16>(d_items, n, maxL, K, S, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_resident_trace(const WorkItem* d_items, int n, int maxL, int K, int S,
                                 hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (maxL > kResidentMaxL) return hipErrorInvalidValue;
  return launch_resident_cls<1024, 16, true>(d_items, n, maxL, K, S, stream);
}

hipError_t launch_put_work(const WorkItem& w, WorkItem* dst, hipStream_t stream) {
  hipLaunchKernelGGL(put_work_kernel, dim3(1), dim3(64), 0, stream, w, dst);
  return hipGetLastError();
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

hipError_t launch_synth(double* x, int64_t L, int n, uint64_t seed, hipStream_t stream) {
  hipLaunchKernelGGL(synth_kernel, dim3(grid_for(L * n, 256)), dim3(256), 0, stream, x, L, n,
                     seed);
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

hipError_t launch_sum_stats(const int64_t* src, int NR, int64_t* dst, hipStream_t stream) {
  hipLaunchKernelGGL(sum_stats_kernel, dim3(1), dim3(64), 0, stream, src, NR, dst);
  return hipGetLastError();
}

hipError_t launch_max_count(const int32_t* n_src, int NR, int32_t* n_out, hipStream_t stream) {
  hipLaunchKernelGGL(max_count_kernel, dim3(1), dim3(64), 0, stream, n_src, NR, n_out);
  return hipGetLastError();
}

hipError_t launch_ceemdan_prep(const CeemdanJob* jobs, int n, int K, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ceemdan_prep_kernel, dim3(n), dim3(kCT), 0, stream, jobs, K);
  return hipGetLastError();
}

hipError_t launch_ceemdan_combine(const CeemdanJob* jobs, int n, int64_t maxL, int stage,
                                  hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int tiles = (int)((maxL + kCTile - 1) / kCTile);
  hipLaunchKernelGGL(ceemdan_combine_kernel, dim3(n, tiles), dim3(kCT), 0, stream, jobs, stage);
  hipLaunchKernelGGL(ceemdan_assess_kernel, dim3(n), dim3(kCT), 0, stream, jobs, stage);
  return hipGetLastError();
}

hipError_t launch_ceemdan_finish(const CeemdanJob* jobs, int n, int K, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ceemdan_finish_kernel, dim3(n, K + 1), dim3(kCT), 0, stream, jobs, K);
  return hipGetLastError();
}

}  // namespace semd
