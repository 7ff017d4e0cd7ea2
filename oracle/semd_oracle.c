/*
 * Serial-EMD CPU oracle -- TEST INFRASTRUCTURE ONLY (parity authority).
 *
 * Plain scalar FP64 C, built with -ffp-contract=off and without fast-math, so
 * every operation below rounds once, in the order written.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use this file; the
 * HIP library never includes, links or calls it, and it uses nothing of the
 * library's.
 *
 * Paper: Zhang, Feng, Marti-Puig, Caiafa, Sun, Duan, Sole-Casals,
 * "Serial-EMD: Fast Empirical Mode Decomposition Method for Multi-dimensional
 * Signals Based on Serialization" (arXiv 2106.15319).
 *
 * Readings taken where the paper is silent (each is listed with its reason in
 * the design notes of the repository):
 *   - extrema: strict neighbours, one extremum at the floor-middle of an
 *     equal-valued run, endpoints and runs touching an endpoint excluded;
 *   - envelopes: natural cubic splines through the extrema plus min(2,n)
 *     knots mirrored about each end sample;
 *   - stopping: S sifts per IMF (earlier if the candidate stops being
 *     siftable); an IMF loop that stops when the residue has no maximum, no
 *     minimum, or fewer than 3 extrema in all, or K IMFs exist;
 *   - outputs: K+1 slots, unused IMF slots zero, residue in slot K
 *     (zero-fill convention of Sec. 4.3);
 *   - EEMD noise: SplitMix64-driven Irwin-Hall normals, added to the
 *     serialized signal (F acts on the serialized x, Sec. 3.3).
 */
#include "semd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Sec. 3.2 -- serialization                                                  */
/* ------------------------------------------------------------------------- */

int64_t semd_ref_serial_length(int64_t M, int64_t N, int64_t D) {
  /* x has (M+D)*N - D = M*N + D*N - D samples (truncation equation). */
  return M * N + D * N - D;
}

int semd_ref_serialize(const double* X, int64_t M, int64_t N, int64_t D, double* x) {
  if (!X || !x || M < 1 || N < 1 || D < 0 || D > M) return -1;
  const int64_t R = M + D; /* rows of T */
  double* a = (double*)malloc(sizeof(double) * (size_t)(D > 0 ? D : 1));
  double* af = (double*)malloc(sizeof(double) * (size_t)(D > 0 ? D : 1));
  double* T = (double*)malloc(sizeof(double) * (size_t)(R * N));
  if (!a || !af || !T) { free(a); free(af); free(T); return -2; }

  /* a_i = i/(D+1), i = 1..D: evenly spaced in (0,1), ends excluded. */
  for (int64_t i = 1; i <= D; ++i) a[i - 1] = (double)i / (double)(D + 1);
  /* a^f: a flipped upside down. */
  for (int64_t i = 0; i < D; ++i) af[i] = a[D - 1 - i];

  /* Upper block of T: X itself. */
  for (int64_t c = 0; c < N; ++c)
    for (int64_t m = 0; m < M; ++m) T[c * R + m] = X[c * M + m];

  /* Lower block of T: E (D x N-1) then the zero column z. */
  for (int64_t c = 0; c < N; ++c) {
    for (int64_t j = 0; j < D; ++j) {
      double e = 0.0;
      if (c < N - 1) {
        /* X_A = X(1:D, 2:N): row j of the flip X_A^f is row D-1-j of X_A,
           i.e. row D-1-j of column c+1 of X (0-based).                     */
        double xa_f = X[(c + 1) * M + (D - 1 - j)];
        /* X_B = X(M-D+1:M, 1:N-1): row j of X_B^f is row D-1-j of X_B,
           i.e. row M-1-j of column c of X (0-based).                        */
        double xb_f = X[c * M + (M - 1 - j)];
        /* E = X_A^f (.) a u^T + X_B^f (.) a^f u^T */
        double p = xa_f * a[j];
        double q = xb_f * af[j];
        e = p + q;
      }
      T[c * R + M + j] = e;
    }
  }
  /* t = vec(T) (column-major), x = t(1 : (M+D)N - D). */
  const int64_t L = semd_ref_serial_length(M, N, D);
  for (int64_t k = 0; k < L; ++k) x[k] = T[k];
  free(a); free(af); free(T);
  return 0;
}

int semd_ref_deserialize(const double* y, int64_t M, int64_t N, int64_t D, double* out) {
  if (!y || !out || M < 1 || N < 1 || D < 0 || D > M) return -1;
  const int64_t R = M + D;
  const int64_t L = semd_ref_serial_length(M, N, D);
  double* T = (double*)malloc(sizeof(double) * (size_t)(R * N));
  if (!T) return -2;
  /* T = [R ; Z]: the serialized result followed by D zeros. */
  for (int64_t k = 0; k < L; ++k) T[k] = y[k];
  for (int64_t k = L; k < R * N; ++k) T[k] = 0.0;
  /* Reshape to (M+D) x N and keep rows 1..M of every column. */
  for (int64_t c = 0; c < N; ++c)
    for (int64_t m = 0; m < M; ++m) out[c * M + m] = T[c * R + m];
  free(T);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1 Step 1 -- extrema                                                 */
/* ------------------------------------------------------------------------- */

int semd_ref_extrema(const double* h, int64_t L, int64_t* imax, int64_t* nmax,
                     int64_t* imin, int64_t* nmin) {
  if (!h || !imax || !imin || !nmax || !nmin || L < 1) return -1;
  int64_t na = 0, ni = 0;
  int64_t k = 0;
  while (k < L) {
    /* maximal run h[k..b] of equal values */
    int64_t b = k;
    while (b + 1 < L && h[b + 1] == h[b]) ++b;
    /* runs touching either end sample are never extrema */
    if (k >= 1 && b <= L - 2) {
      int64_t mid = (k + b) / 2; /* floor of the run's middle */
      if (h[k - 1] < h[k] && h[b + 1] < h[b]) imax[na++] = mid;
      else if (h[k - 1] > h[k] && h[b + 1] > h[b]) imin[ni++] = mid;
    }
    k = b + 1;
  }
  *nmax = na;
  *nmin = ni;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1 Step 2 -- natural cubic spline envelopes                          */
/* ------------------------------------------------------------------------- */

int semd_ref_spline_solve(const double* t, const double* y, int64_t n, double* Mpp) {
  if (!t || !y || !Mpp || n < 3) return -1;
  for (int64_t j = 0; j + 1 < n; ++j)
    if (!(t[j + 1] > t[j])) return -1;
  /* Natural end conditions. */
  Mpp[0] = 0.0;
  Mpp[n - 1] = 0.0;
  const int64_t m = n - 2; /* interior unknowns Mpp[1..n-2] */
  double* cp = (double*)malloc(sizeof(double) * (size_t)m);
  double* dp = (double*)malloc(sizeof(double) * (size_t)m);
  if (!cp || !dp) { free(cp); free(dp); return -2; }
  /* Row j (1 <= j <= n-2):
       g_{j-1} M_{j-1} + 2 (g_{j-1} + g_j) M_j + g_j M_{j+1}
         = 6 ((y_{j+1} - y_j)/g_j - (y_j - y_{j-1})/g_{j-1})
     Thomas algorithm: forward elimination, then back substitution. */
  for (int64_t j = 1; j <= n - 2; ++j) {
    double g0 = t[j] - t[j - 1];
    double g1 = t[j + 1] - t[j];
    double s1 = (y[j + 1] - y[j]) / g1;
    double s0 = (y[j] - y[j - 1]) / g0;
    double rhs = 6.0 * (s1 - s0);
    double diag = 2.0 * (g0 + g1);
    double sub = g0, sup = g1;
    int64_t i = j - 1;
    if (i == 0) {
      cp[i] = sup / diag;
      dp[i] = rhs / diag;
    } else {
      double den = diag - sub * cp[i - 1];
      cp[i] = sup / den;
      dp[i] = (rhs - sub * dp[i - 1]) / den;
    }
  }
  Mpp[m] = dp[m - 1];
  for (int64_t i = m - 2; i >= 0; --i) Mpp[i + 1] = dp[i] - cp[i] * Mpp[i + 2];
  free(cp); free(dp);
  return 0;
}

int semd_ref_spline_eval(const double* t, const double* y, const double* Mpp,
                         int64_t n, int64_t L, double* out) {
  if (!t || !y || !Mpp || !out || n < 2 || L < 1) return -1;
  if (!(t[0] <= 0.0) || !(t[n - 1] >= (double)(L - 1))) return -1;
  int64_t j = 0;
  for (int64_t k = 0; k < L; ++k) {
    double kk = (double)k;
    /* segment j: t[j] <= k < t[j+1] (j = number of knots <= k, minus one) */
    while (j + 2 < n && t[j + 1] <= kk) ++j;
    double g = t[j + 1] - t[j];
    double A = t[j + 1] - kk;
    double B = kk - t[j];
    double A3 = A * A * A;
    double B3 = B * B * B;
    double g2 = g * g;
    double cub = (Mpp[j] * A3 + Mpp[j + 1] * B3) / (6.0 * g);
    double lin = (y[j] - Mpp[j] * g2 / 6.0) * A / g + (y[j + 1] - Mpp[j + 1] * g2 / 6.0) * B / g;
    out[k] = cub + lin;
  }
  return 0;
}

int semd_ref_envelope(const double* h, int64_t L, const int64_t* idx, int64_t n, double* env) {
  if (!h || !idx || !env || n < 1 || L < 3) return -1;
  /* Mirror boundary: P = min(2, n) knots reflected about sample 0 and about
     sample L-1, carrying the value of their source extremum. */
  const int64_t P = n < 2 ? n : 2;
  const int64_t nk = n + 2 * P;
  double* t = (double*)malloc(sizeof(double) * (size_t)nk);
  double* y = (double*)malloc(sizeof(double) * (size_t)nk);
  double* M2 = (double*)malloc(sizeof(double) * (size_t)nk);
  if (!t || !y || !M2) { free(t); free(y); free(M2); return -2; }
  int64_t q = 0;
  for (int64_t p = P - 1; p >= 0; --p) { t[q] = -(double)idx[p]; y[q] = h[idx[p]]; ++q; }
  for (int64_t p = 0; p < n; ++p) { t[q] = (double)idx[p]; y[q] = h[idx[p]]; ++q; }
  for (int64_t p = n - 1; p >= n - P; --p) {
    t[q] = (double)(2 * (L - 1) - idx[p]);
    y[q] = h[idx[p]];
    ++q;
  }
  int rc = semd_ref_spline_solve(t, y, nk, M2);
  if (rc == 0) rc = semd_ref_spline_eval(t, y, M2, nk, L, env);
  free(t); free(y); free(M2);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.1 Steps 1-5 -- sifting and the IMF loop                             */
/* ------------------------------------------------------------------------- */

static int siftable(int64_t nmax, int64_t nmin) {
  return nmax >= 1 && nmin >= 1 && nmax + nmin >= 3;
}

static void note_gaps(const double* h, int64_t L, semd_ref_stats* st) {
  for (int64_t k = 0; k + 1 < L; ++k) {
    double d = fabs(h[k + 1] - h[k]);
    if (d == 0.0) st->n_equal += 1;
    else if (d < st->min_gap) st->min_gap = d;
  }
}

/* Where a traced decomposition writes its extremum decisions (see
 * semd_ref_emd_trace); NULL for an untraced one. */
typedef struct {
  int64_t* buf;
  int64_t cap, used;
  int complete;
  int want_imf, want_sift;
  double* h_at;
  int found;
} trace_ctx;

/* One detection: the record (imf, sift, counts, index lists), and the tested
 * array itself when it is the one asked for. */
static void trace_detection(trace_ctx* tc, int imf, int sift, const double* tested, int64_t L,
                            const int64_t* imax, int64_t na, const int64_t* imin, int64_t ni) {
  if (!tc) return;
  if (tc->h_at && imf == tc->want_imf && sift == tc->want_sift) {
    memcpy(tc->h_at, tested, sizeof(double) * (size_t)L);
    tc->found = 1;
  }
  if (!tc->buf || !tc->complete) return;
  const int64_t need = 4 + na + ni;
  if (tc->used + need > tc->cap) {
    tc->complete = 0;
    return;
  }
  int64_t* o = tc->buf + tc->used;
  o[0] = imf;
  o[1] = sift;
  o[2] = na;
  o[3] = ni;
  for (int64_t j = 0; j < na; ++j) o[4 + j] = imax[j];
  for (int64_t j = 0; j < ni; ++j) o[4 + na + j] = imin[j];
  tc->used += need;
}

static int emd_core(const double* x, int64_t L, int K, int S, double sd_threshold,
                    double* imfs, int* n_imfs, semd_ref_stats* stats, trace_ctx* tc);

int semd_ref_emd(const double* x, int64_t L, int K, int S, double* imfs, int* n_imfs,
                 semd_ref_stats* stats) {
  return emd_core(x, L, K, S, 0.0, imfs, n_imfs, stats, NULL);
}

int semd_ref_emd_sd(const double* x, int64_t L, int K, int S, double sd_threshold,
                    double* imfs, int* n_imfs, semd_ref_stats* stats) {
  return emd_core(x, L, K, S, sd_threshold, imfs, n_imfs, stats, NULL);
}

int semd_ref_emd_trace(const double* x, int64_t L, int K, int S, double sd_threshold,
                       double* imfs, int* n_imfs, int64_t* buf, int64_t cap, int64_t* used,
                       int* complete, int want_imf, int want_sift, double* h_at, int* found) {
  if (!used || !complete || (cap > 0 && !buf) || cap < 0) return -1;
  trace_ctx tc = {buf, cap, 0, 1, want_imf, want_sift, h_at, 0};
  const int rc = emd_core(x, L, K, S, sd_threshold, imfs, n_imfs, NULL, &tc);
  *used = tc.used;
  *complete = tc.complete;
  if (found) *found = tc.found;
  return rc;
}

static int emd_core(const double* x, int64_t L, int K, int S, double sd_threshold,
                    double* imfs, int* n_imfs, semd_ref_stats* stats, trace_ctx* tc) {
  if (!x || !imfs || !n_imfs || L < 1 || K < 1 || S < 1 || !(sd_threshold >= 0.0)) return -1;
  for (int64_t k = 0; k < L; ++k)
    if (!isfinite(x[k])) return -3;
  semd_ref_stats st;
  st.min_gap = INFINITY;
  st.n_sifts = 0;
  st.n_equal = 0;
  st.sd_margin = INFINITY;

  const size_t nb = sizeof(double) * (size_t)L;
  double* r = (double*)malloc(nb);
  double* h = (double*)malloc(nb);
  double* up = (double*)malloc(nb);
  double* lo = (double*)malloc(nb);
  int64_t* imax = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L / 2 + 2));
  int64_t* imin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L / 2 + 2));
  if (!r || !h || !up || !lo || !imax || !imin) {
    free(r); free(h); free(up); free(lo); free(imax); free(imin);
    return -2;
  }
  memset(imfs, 0, sizeof(double) * (size_t)(K + 1) * (size_t)L);
  memcpy(r, x, nb);
  int pristine = 1; /* r still equals the input: its extremum tests are exact */
  int nimf = 0;
  int rc = 0;
  while (nimf < K) {
    int64_t na, ni;
    if (L < 3) break;
    if (!pristine) note_gaps(r, L, &st);
    semd_ref_extrema(r, L, imax, &na, imin, &ni);
    trace_detection(tc, nimf, 0, r, L, imax, na, imin, ni);
    if (!siftable(na, ni)) break;
    memcpy(h, r, nb); /* h = r */
    for (int s = 0; s < S; ++s) {
      if (s > 0) {
        note_gaps(h, L, &st);
        semd_ref_extrema(h, L, imax, &na, imin, &ni);
        trace_detection(tc, nimf, s, h, L, imax, na, imin, ni);
        if (!siftable(na, ni)) break;
      }
      /* Step 2: upper and lower envelopes; Step 3: local mean;
         Step 4: candidate s = h - m. */
      rc = semd_ref_envelope(h, L, imax, na, up);
      if (rc == 0) rc = semd_ref_envelope(h, L, imin, ni, lo);
      if (rc != 0) goto done;
      /* the change of this sift is the mean m itself: SD = sum m^2 / sum h^2
         over the candidate before the sift (Huang et al. 1998) */
      double num = 0.0, den = 0.0;
      for (int64_t k = 0; k < L; ++k) {
        double m = 0.5 * (up[k] + lo[k]);
        num += m * m;
        den += h[k] * h[k];
        h[k] = h[k] - m;
      }
      pristine = 0;
      st.n_sifts += 1;
      if (sd_threshold > 0.0 && s + 1 < S) {
        const double lim = sd_threshold * den;
        if (lim > 0.0) {
          const double margin = fabs(num - lim) / lim;
          if (margin < st.sd_margin) st.sd_margin = margin;
        }
        if (num < lim) break;
      }
    }
    /* Step 5 (fixed-count criterion): c_i = h; residue r = r - c_i. */
    memcpy(imfs + (size_t)nimf * (size_t)L, h, nb);
    for (int64_t k = 0; k < L; ++k) r[k] = r[k] - h[k];
    nimf += 1;
  }
  memcpy(imfs + (size_t)K * (size_t)L, r, nb);
  *n_imfs = nimf;
  if (stats) *stats = st;
done:
  free(r); free(h); free(up); free(lo); free(imax); free(imin);
  return rc;
}

int semd_ref_decompose(const double* X, int64_t M, int64_t N, int64_t D, int K, int S,
                       double* out, int* n_imfs, semd_ref_stats* stats) {
  return semd_ref_decompose_sd(X, M, N, D, K, S, 0.0, out, n_imfs, stats);
}

int semd_ref_decompose_sd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S,
                          double sd_threshold, double* out, int* n_imfs, semd_ref_stats* stats) {
  if (!X || !out || !n_imfs || M < 1 || N < 1 || D < 0 || D > M || K < 1 || S < 1) return -1;
  const int64_t L = semd_ref_serial_length(M, N, D);
  double* x = (double*)malloc(sizeof(double) * (size_t)L);
  double* R = (double*)malloc(sizeof(double) * (size_t)L * (size_t)(K + 1));
  if (!x || !R) { free(x); free(R); return -2; }
  int rc = semd_ref_serialize(X, M, N, D, x);
  if (rc == 0) rc = semd_ref_emd_sd(x, L, K, S, sd_threshold, R, n_imfs, stats);
  if (rc == 0)
    for (int k = 0; k <= K; ++k)
      semd_ref_deserialize(R + (size_t)k * (size_t)L, M, N, D, out + (size_t)k * (size_t)(M * N));
  free(x); free(R);
  return rc;
}

int semd_ref_decompose_slices(const double* X, int64_t M, int64_t N, int K, int S,
                              double* out, int* n_imfs) {
  return semd_ref_decompose_slices_sd(X, M, N, K, S, 0.0, out, n_imfs);
}

int semd_ref_decompose_slices_sd(const double* X, int64_t M, int64_t N, int K, int S,
                                 double sd_threshold, double* out, int* n_imfs) {
  if (!X || !out || !n_imfs || M < 1 || N < 1 || K < 1 || S < 1) return -1;
  double* R = (double*)malloc(sizeof(double) * (size_t)M * (size_t)(K + 1));
  if (!R) return -2;
  int rc = 0;
  for (int64_t c = 0; c < N && rc == 0; ++c) {
    rc = semd_ref_emd_sd(X + c * M, M, K, S, sd_threshold, R, &n_imfs[c], NULL);
    for (int k = 0; k <= K && rc == 0; ++k)
      memcpy(out + (size_t)k * (size_t)(M * N) + (size_t)(c * M), R + (size_t)k * (size_t)M,
             sizeof(double) * (size_t)M);
  }
  free(R);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2 -- EEMD                                                           */
/* ------------------------------------------------------------------------- */

uint64_t semd_ref_splitmix64(uint64_t state, uint64_t n) {
  /* The generator adds the odd constant gamma (the 64-bit golden ratio) to its
     state at every call and returns a bijective mix of the new state. */
  uint64_t z = state + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int semd_ref_noise(uint64_t seed, uint64_t item, uint64_t m, int64_t L, double* w) {
  if (!w || L < 0) return -1;
  /* One stream per (seed, item, realization). */
  uint64_t s1 = semd_ref_splitmix64(seed, item + 1);
  uint64_t s2 = semd_ref_splitmix64(s1, m + 1);
  for (int64_t k = 0; k < L; ++k) {
    /* 12 uniforms on the 2^-53 grid, summed exactly as integers. */
    uint64_t acc = 0;
    for (uint64_t j = 0; j < 12; ++j)
      acc += semd_ref_splitmix64(s2, 12ull * (uint64_t)k + j + 1) >> 11;
    int64_t c = (int64_t)acc - (int64_t)(6ull << 53);
    w[k] = (double)c * 0x1p-53; /* one rounding, then an exact scale */
  }
  return 0;
}

int semd_ref_eemd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                  double beta, uint64_t seed, uint64_t item, double* out) {
  return semd_ref_eemd_sd(X, M, N, D, K, S, NR, beta, seed, item, 0.0, out);
}

int semd_ref_eemd_sd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                     double beta, uint64_t seed, uint64_t item, double sd_threshold,
                     double* out) {
  if (!X || !out || M < 1 || N < 1 || D < 0 || D > M || K < 1 || S < 1 || NR < 1) return -1;
  if (!isfinite(beta)) return -1;
  const int64_t L = semd_ref_serial_length(M, N, D);
  const size_t slot = (size_t)L;
  double* x = (double*)malloc(sizeof(double) * slot);
  double* xm = (double*)malloc(sizeof(double) * slot);
  double* w = (double*)malloc(sizeof(double) * slot);
  double* R = (double*)malloc(sizeof(double) * slot * (size_t)(K + 1));
  double* acc = (double*)calloc(slot * (size_t)(K + 1), sizeof(double));
  if (!x || !xm || !w || !R || !acc) {
    free(x); free(xm); free(w); free(R); free(acc);
    return -2;
  }
  int rc = semd_ref_serialize(X, M, N, D, x);
  for (int m = 0; m < NR && rc == 0; ++m) {
    /* Step 1: x_m = x + beta w_m */
    semd_ref_noise(seed, item, (uint64_t)m, L, w);
    for (int64_t k = 0; k < L; ++k) {
      double bw = beta * w[k];
      xm[k] = x[k] + bw;
    }
    /* Step 2: decompose each x_m completely by EMD */
    int nimf = 0;
    rc = semd_ref_emd_sd(xm, L, K, S, sd_threshold, R, &nimf, NULL);
    /* Step 3 (accumulate in realization order, zero slots included) */
    for (size_t i = 0; rc == 0 && i < slot * (size_t)(K + 1); ++i) acc[i] = acc[i] + R[i];
  }
  if (rc == 0) {
    for (size_t i = 0; i < slot * (size_t)(K + 1); ++i) acc[i] = acc[i] / (double)NR;
    for (int k = 0; k <= K; ++k)
      semd_ref_deserialize(acc + (size_t)k * slot, M, N, D, out + (size_t)k * (size_t)(M * N));
  }
  free(x); free(xm); free(w); free(R); free(acc);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2 -- CEEMDAN                                                        */
/* ------------------------------------------------------------------------- */

/* Population standard deviation of v[0..L): mean, then the mean squared
   deviation, both summed in index order. */
static double pop_std(const double* v, int64_t L) {
  double s = 0.0;
  for (int64_t k = 0; k < L; ++k) s = s + v[k];
  const double mean = s / (double)L;
  double q = 0.0;
  for (int64_t k = 0; k < L; ++k) {
    const double d = v[k] - mean;
    q = q + d * d;
  }
  return sqrt(q / (double)L);
}

static int is_siftable(const double* v, int64_t L, int64_t* imax, int64_t* imin) {
  int64_t na = 0, ni = 0;
  if (L < 3) return 0;
  semd_ref_extrema(v, L, imax, &na, imin, &ni);
  return siftable(na, ni);
}

int semd_ref_ceemdan(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                     double eps, uint64_t seed, uint64_t item, double sd_threshold,
                     double* out, int* n_modes) {
  if (!X || !out || !n_modes || M < 1 || N < 1 || D < 0 || D > M || K < 1 || S < 1 || NR < 1)
    return -1;
  if (!isfinite(eps) || eps < 0.0 || !(sd_threshold >= 0.0)) return -1;
  const int64_t L = semd_ref_serial_length(M, N, D);
  const size_t nb = sizeof(double) * (size_t)L;
  double* r = (double*)malloc(nb);
  double* v = (double*)malloc(nb);
  double* acc = (double*)malloc(nb);
  double* modes = (double*)calloc((size_t)K * (size_t)L, sizeof(double));
  double* E = (double*)malloc(nb * (size_t)NR * (size_t)(K + 1));  /* E[m] = EMD(w_m) */
  double* F = (double*)malloc(nb * 2);                              /* one first mode */
  int64_t* imax = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L / 2 + 2));
  int64_t* imin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L / 2 + 2));
  if (!r || !v || !acc || !modes || !E || !F || !imax || !imin) {
    free(r); free(v); free(acc); free(modes); free(E); free(F); free(imax); free(imin);
    return -2;
  }
  int rc = semd_ref_serialize(X, M, N, D, r); /* r_0 = x */
  for (int64_t k = 0; k < L && rc == 0; ++k)
    if (!isfinite(r[k])) rc = -3;
  /* E_i(w_m): the i-th mode of the EMD of noise realization m (zero if it
     has fewer modes), i = 1..K; kept as slot i-1 of E[m]. */
  for (int m = 0; m < NR && rc == 0; ++m) {
    int nm = 0;
    semd_ref_noise(seed, item, (uint64_t)m, L, v);
    rc = semd_ref_emd_sd(v, L, K, S, sd_threshold, E + (size_t)m * (size_t)(K + 1) * (size_t)L,
                         &nm, NULL);
  }
  int n = 0;
  for (int i = 1; i <= K && rc == 0; ++i) {
    /* stage i extracts mode i from r_{i-1}, if r_{i-1} can still be sifted */
    if (!is_siftable(r, L, imax, imin)) break;
    const double beta = eps * pop_std(r, L);
    for (int64_t k = 0; k < L; ++k) acc[k] = 0.0;
    for (int m = 0; m < NR && rc == 0; ++m) {
      /* stage 1 adds beta_0 w_m (the EEMD step); stage i > 1 adds
         beta_{i-1} E_{i-1}(w_m) */
      if (i == 1) semd_ref_noise(seed, item, (uint64_t)m, L, v);
      const double* e = (i == 1) ? v : E + ((size_t)m * (size_t)(K + 1) + (size_t)(i - 2)) * (size_t)L;
      for (int64_t k = 0; k < L; ++k) {
        const double be = beta * e[k];
        v[k] = r[k] + be;
      }
      int nm = 0;
      rc = semd_ref_emd_sd(v, L, 1, S, sd_threshold, F, &nm, NULL); /* first mode of v */
      for (int64_t k = 0; k < L && rc == 0; ++k) acc[k] = acc[k] + F[k];
    }
    if (rc) break;
    double* c = modes + (size_t)(i - 1) * (size_t)L;
    for (int64_t k = 0; k < L; ++k) {
      c[k] = acc[k] / (double)NR; /* the i-th CEEMDAN mode */
      r[k] = r[k] - c[k];         /* r_i = r_{i-1} - c_i */
    }
    n = i;
  }
  if (rc == 0) {
    const int64_t MN = M * N;
    for (int i = 0; i < K; ++i)
      semd_ref_deserialize(modes + (size_t)i * (size_t)L, M, N, D, out + (size_t)i * (size_t)MN);
    semd_ref_deserialize(r, M, N, D, out + (size_t)K * (size_t)MN);
    *n_modes = n;
  }
  free(r); free(v); free(acc); free(modes); free(E); free(F); free(imax); free(imin);
  return rc;
}
