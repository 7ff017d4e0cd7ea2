/*
 * Serial-EMD CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar FP64 implementation of what the Serial-EMD hot path
 * computes (Zhang et al., "Serial-EMD: Fast Empirical Mode Decomposition Method
 * for Multi-dimensional Signals Based on Serialization", arXiv 2106.15319).
 * It is the parity authority for the HIP library and is used only by the
 * tests, the smoke check and the CPU-baseline leg of the benchmark.  It shares
 * no code with the HIP library (no header, helper, table or generator).
 *
 * All pointers are host memory.  All arrays are plain C arrays of doubles
 * (or int64 for indices).  Functions return 0 on success, a negative value on
 * invalid arguments.  Nothing here allocates memory it does not free.
 *
 * Layout: X is M x N column-major (fibre i = column i, element (m,i) at m+M*i),
 * as in Sec. 3.2 (the signals are the columns of X).
 */
#ifndef SEMD_ORACLE_H
#define SEMD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sec. 3.2, final truncation: length of the serialized signal, M*N + D*N - D. */
int64_t semd_ref_serial_length(int64_t M, int64_t N, int64_t D);

/* Sec. 3.2 (vector a, sub-matrices X_A and X_B, transitions E, block matrix T,
 * vec(T), truncation).  X: M*N doubles; x: serial_length doubles. */
int semd_ref_serialize(const double* X, int64_t M, int64_t N, int64_t D, double* x);

/* Sec. 3.3 (append D zeros, reshape to (M+D) x N, keep rows 1..M).
 * y: serial_length doubles; out: M*N doubles. */
int semd_ref_deserialize(const double* y, int64_t M, int64_t N, int64_t D, double* out);

/* Sec. 2.1 Step 1: local maxima / minima of h (plateau-middle rule, endpoints
 * excluded).  Index lists are written in increasing order; imax and imin must
 * hold at least L/2+1 entries each. */
int semd_ref_extrema(const double* h, int64_t L, int64_t* imax, int64_t* nmax,
                     int64_t* imin, int64_t* nmin);

/* Natural cubic spline through (t[j], y[j]), j<n, n>=3, t strictly increasing:
 * second derivatives Mpp[j] (Mpp[0] = Mpp[n-1] = 0) by the Thomas algorithm. */
int semd_ref_spline_solve(const double* t, const double* y, int64_t n, double* Mpp);

/* Evaluate that spline at the integers k = 0..L-1 (t[0] < 0 <= L-1 < t[n-1]). */
int semd_ref_spline_eval(const double* t, const double* y, const double* Mpp,
                         int64_t n, int64_t L, double* out);

/* Sec. 2.1 Step 2: envelope of h through the extrema idx[0..n-1] (n>=1), with
 * min(2,n) mirrored knots per end; env: L doubles. */
int semd_ref_envelope(const double* h, int64_t L, const int64_t* idx, int64_t n, double* env);

/* Decision statistics of one decomposition, for the tie-aware comparison. */
typedef struct {
  double min_gap;      /* min |h[k+1]-h[k]| over every adjacent unequal pair   */
                       /* seen by an extremum test after the very first one   */
  int64_t n_sifts;     /* sifts performed                                      */
  int64_t n_equal;     /* adjacent equal pairs seen after the first test       */
  double sd_margin;    /* min |num - thr*den| / (thr*den) over the SD tests    */
                       /* that could end an IMF early (INFINITY if none)      */
} semd_ref_stats;

/* Sec. 2.1 Steps 1-5 with a fixed number S of sifts per IMF and at most K IMFs.
 * imfs: (K+1)*L doubles; slot k < *n_imfs = IMF k, slots *n_imfs..K-1 = 0,
 * slot K = residue.  stats may be NULL. */
int semd_ref_emd(const double* x, int64_t L, int K, int S, double* imfs, int* n_imfs,
                 semd_ref_stats* stats);

/* Sec. 2.1 with a data-dependent stop (Step 5 leaves the criterion open): as
 * semd_ref_emd, but an IMF also ends after the sift whose mean m satisfies
 * sum_k m[k]^2 < sd_threshold * sum_k h[k]^2, h the candidate before that
 * sift (a standard-deviation test between consecutive candidates in its
 * ratio-of-sums, Cauchy-type form, since h - (h - m) = m; both sums taken in
 * k order), with at most S sifts.  sd_threshold = 0 is the fixed-count
 * rule. */
int semd_ref_emd_sd(const double* x, int64_t L, int K, int S, double sd_threshold,
                    double* imfs, int* n_imfs, semd_ref_stats* stats);

/* semd_ref_emd_sd with its extremum decisions recorded (Sec. 2.1 Step 1), for
 * the per-sift parity comparison.  Every detection the loop makes -- on the
 * residue before IMF i (sift index 0) and on the candidate before sift s > 0
 * of IMF i -- appends the record
 *   i, s, nmax, nmin, maxima (nmax indices), minima (nmin indices)
 * to buf while the whole record fits in cap entries; *used receives the
 * entries written, *complete 0 once a record did not fit.  When h_at is not
 * NULL, the array tested by detection (want_imf, want_sift) is copied there
 * (L doubles) and *found (if not NULL) set to 1, else to 0. */
int semd_ref_emd_trace(const double* x, int64_t L, int K, int S, double sd_threshold,
                       double* imfs, int* n_imfs, int64_t* buf, int64_t cap, int64_t* used,
                       int* complete, int want_imf, int want_sift, double* h_at, int* found);

/* Serial-EMD: serialize (Sec. 3.2), EMD (Sec. 2.1), deserialize (Sec. 3.3).
 * out: (K+1)*M*N doubles in the same slot convention. */
int semd_ref_decompose(const double* X, int64_t M, int64_t N, int64_t D, int K, int S,
                       double* out, int* n_imfs, semd_ref_stats* stats);

/* semd_ref_decompose with the SD stopping rule of semd_ref_emd_sd. */
int semd_ref_decompose_sd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S,
                          double sd_threshold, double* out, int* n_imfs,
                          semd_ref_stats* stats);

/* Standard-version (slice-wise) EMD: every column of X decomposed on its own,
 * no serialization (Sec. 4 opening).  out: (K+1)*M*N; n_imfs: N ints. */
int semd_ref_decompose_slices(const double* X, int64_t M, int64_t N, int K, int S,
                              double* out, int* n_imfs);
/* The same with the SD stopping rule of semd_ref_emd_sd. */
int semd_ref_decompose_slices_sd(const double* X, int64_t M, int64_t N, int K, int S,
                                 double sd_threshold, double* out, int* n_imfs);

/* SplitMix64 (Steele, Lea & Flood 2014): the n-th output (n >= 1) of the
 * generator whose state starts at `state`. */
uint64_t semd_ref_splitmix64(uint64_t state, uint64_t n);

/* White noise for EEMD realization m of item `item`: L samples, each the
 * Irwin-Hall sum of 12 uniforms minus 6 (zero mean, unit variance). */
int semd_ref_noise(uint64_t seed, uint64_t item, uint64_t m, int64_t L, double* w);

/* Sec. 2.2 EEMD on the serialized signal: x_m = x + beta*w_m for m < NR,
 * EMD of each, slot-wise mean over m (zero slots included).  beta is absolute.
 * out: (K+1)*M*N doubles (mean IMFs, mean residue in slot K). */
int semd_ref_eemd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                  double beta, uint64_t seed, uint64_t item, double* out);
/* The same with the SD stopping rule of semd_ref_emd_sd in every realization. */
int semd_ref_eemd_sd(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                     double beta, uint64_t seed, uint64_t item, double sd_threshold,
                     double* out);

/* Sec. 2.2 CEEMDAN (Torres et al. 2011) on the serialized signal x.  With
 * w_m the noise realization m of semd_ref_noise (m < NR), E_i(w) the i-th
 * mode of the EMD of w (zero if it has fewer), F1(v) the first mode of the
 * EMD of v and std the population standard deviation:
 *   stage 1:      c_1 = mean_m F1(x + beta_0 w_m),               beta_0 = eps std(x)
 *   stage i > 1:  c_i = mean_m F1(r_{i-1} + beta_{i-1} E_{i-1}(w_m)),
 *                                                    beta_{i-1} = eps std(r_{i-1})
 *   r_i = r_{i-1} - c_i (r_0 = x); a stage runs only while r_{i-1} is siftable
 *   and i <= K.  Every EMD uses S sifts per mode and the SD rule when
 *   sd_threshold > 0.  out: (K+1)*M*N doubles, modes 0..n-1, zeros, residue
 *   in slot K; *n_modes = n. */
int semd_ref_ceemdan(const double* X, int64_t M, int64_t N, int64_t D, int K, int S, int NR,
                     double eps, uint64_t seed, uint64_t item, double sd_threshold,
                     double* out, int* n_modes);

#ifdef __cplusplus
}
#endif
#endif
