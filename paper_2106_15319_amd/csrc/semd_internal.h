// Internal interfaces between the C ABI layer (semd_api.hip) and the kernels
// (semd_kernels.hip).  Not installed; callers use include/semd.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace semd {

// One unit of resident-path work: one serialized signal (optionally one EEMD
// realization of it) decomposed by one workgroup.
struct WorkItem {
  const double* X;   // device, M*N column-major input
  double* out;       // device, (K+1)*M*N output slots
  int32_t* n_imfs;   // device, one int32 or nullptr
  int64_t* stats;    // device, 3 int64 (sifts, knots, sample-sifts) or nullptr
  double* r;         // device workspace, L doubles (residue, serialized)
  double* u;         // device workspace, resident_ws_doubles(L) - L doubles: the
                     // parked upper envelope, or the global knot store
  int64_t M;         // fibre length (rows of X)
  int64_t N;         // number of fibres (columns of X)
  int32_t D;         // transition length
  int32_t L;         // serialized length M*N + D*N - D
  double beta;       // EEMD noise amplitude
  uint64_t key;      // SplitMix64 stream key of this realization
  int32_t flags;     // kAddNoise | kAddBuffer | kScaleOnDevice | kNoSignal
  int32_t pad;
  int64_t slot_stride;  // doubles from one output slot to the next (M*N when contiguous)
  double sd;         // SD stopping threshold; 0: fixed sift count
  const double* addend;  // device, L doubles added (scaled) under kAddBuffer
  const double* scale;   // device, one double replacing beta under kScaleOnDevice
  int32_t* trace;        // device, trace_cap int32: extremum decisions, or nullptr
  int32_t trace_cap;
  int32_t pad2;
};

// What the first load adds to the serialized signal x (Sec. 2.2):
//   kAddNoise       x + b * w, w the realization's white noise (key);
//   kAddBuffer      x + b * addend;
//   kScaleOnDevice  b = *scale (else b = beta);
//   kNoSignal       x = 0 (the input is not read).
constexpr int32_t kAddNoise = 1, kAddBuffer = 2, kScaleOnDevice = 4, kNoSignal = 8;

// Longest serialized signal the resident kernel handles (threads x samples
// per thread of its largest instance).
constexpr int kResidentMaxL = 16384;

// Knots the global knot store of one resident item holds: both envelopes of
// any sift (at most L - 2 extrema plus 8 mirrored knots).
__host__ __device__ constexpr int resident_gknot_cap(int L) { return L + 16; }

// Workspace doubles of one resident item: the residue (L) and the region u,
// which holds either the parked upper envelope (L doubles) or the global knot
// store (4 doubles and one int16 per knot).
__host__ __device__ constexpr int64_t resident_ws_doubles(int64_t L) {
  return L + 4 * (L + 16) + ((L + 16) * 2 + 7) / 8 + 2;
}

// Launch shape of the resident kernel: threads per workgroup and samples per
// thread.  resident_class() is the default choice for the longest signal of a
// launch of few signals (regime 0) or of at least one per compute unit
// (regime 1); a tuned table may choose another.
struct ResidentClass {
  int nt;
  int c;
};
ResidentClass resident_class(int maxL, int regime);

// Bytes of the kernel's reusable LDS area (staging window, knot store) for
// signals up to maxL samples, at most max_area (and at least what the
// staging window needs).
size_t resident_area_bytes(int maxL, int nt, size_t max_area);

// The compiled launch shapes: up to cap of them into out; returns how many
// exist.
int resident_classes(ResidentClass* out, int cap);

// Launch the resident kernel with shape c (c.nt * c.c >= maxL) over `n` work
// items (device array), all with L <= maxL.  Returns hipSuccess or the
// launch error (hipErrorInvalidValue for a shape that is not compiled).
hipError_t launch_resident(const WorkItem* d_items, int n, int maxL, ResidentClass c, int K,
                           int S, hipStream_t stream);

// Write the descriptor w to device memory dst (stream-ordered, by a kernel:
// no host staging buffer and no allocation).
hipError_t launch_put_work(const WorkItem& w, WorkItem* dst, hipStream_t stream);

// The resident kernel with every extremum detection recorded in each item's
// trace (launch shape 1024 threads x 16 samples, any L <= kResidentMaxL):
// trace[0] entries used (4 header entries included), trace[1] 1 while every
// record fitted, then one record per detection: imf, sift, nmax, nmin, the
// maxima's and the minima's positions in increasing order.
hipError_t launch_resident_trace(const WorkItem* d_items, int n, int maxL, int K, int S,
                                 hipStream_t stream);

// Extrema of one 1D signal (3 <= L <= kResidentMaxL) through the resident
// detection/compaction code: indices to imax/imin, counts[0..1].
hipError_t launch_extrema(const double* h, int L, int32_t* imax, int32_t* imin,
                          int32_t* counts, hipStream_t stream);

hipError_t launch_serialize(const double* X, int64_t M, int64_t N, int D, double* x,
                            hipStream_t stream);
hipError_t launch_deserialize(const double* y, int64_t M, int64_t N, int D, double* out,
                              hipStream_t stream);
hipError_t launch_noise(uint64_t key, int64_t L, double* w, hipStream_t stream);
// Synthetic tuning signals: n x L doubles at x (two sinusoids and noise).
hipError_t launch_synth(double* x, int64_t L, int n, uint64_t seed, hipStream_t stream);

// Slot-wise mean over NR realization buffers: src holds NR consecutive blocks
// of `count` doubles; dst[i] = (sum_m src[m*count + i]) / NR, summed in m order.
hipError_t launch_ensemble_mean(const double* src, int NR, int64_t count, double* dst,
                                hipStream_t stream);
// n_out[0] = max over m of n_src[m] (error codes, negative, take precedence).
hipError_t launch_max_count(const int32_t* n_src, int NR, int32_t* n_out, hipStream_t stream);
// dst[0..2] = sums over m < NR of src[3m .. 3m+2] (work statistics).
hipError_t launch_sum_stats(const int64_t* src, int NR, int64_t* dst, hipStream_t stream);

// CEEMDAN (Sec. 2.2) per-item state and buffers, all device memory.
struct CeemdanState {
  double scale;   // beta of the next stage: eps * std of the current residue
  int32_t alive;  // the current residue can still be sifted
  int32_t n;      // modes extracted (-5: the input holds NaN/Inf)
};
struct CeemdanJob {
  double* r;              // residue, L doubles (serialized domain)
  double* modes;          // K x L mode slots (serialized domain)
  const double* stage;    // NR x 2L: the stage's first modes (slot 0 of each)
  double* out;            // (K+1) output slots, slot_stride apart (deserialized)
  int32_t* n_out;         // or nullptr
  CeemdanState* st;
  int64_t M, N, L, slot_stride;
  int32_t D, NR;
  double eps;
};
// Zero the mode slots, mark non-finite input, and set the first stage's
// state from r = x.
hipError_t launch_ceemdan_prep(const CeemdanJob* jobs, int n, int K, hipStream_t stream);
// Stage `stage` (1-based): mean of the NR first modes into mode slot
// stage-1 and r -= mode (if alive); then alive and scale from the new r.
// maxL: the longest item.
hipError_t launch_ceemdan_combine(const CeemdanJob* jobs, int n, int64_t maxL, int stage,
                                  hipStream_t stream);
// Deserialize the modes and residue into the outputs; mode count.
hipError_t launch_ceemdan_finish(const CeemdanJob* jobs, int n, int K, hipStream_t stream);

// SplitMix64: n-th output of the generator started at `state`.
__host__ __device__ inline uint64_t splitmix64(uint64_t state, uint64_t n) {
  uint64_t z = state + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Stream key of realization m of item `item` under `seed`.
__host__ __device__ inline uint64_t noise_key(uint64_t seed, uint64_t item, uint64_t m) {
  return splitmix64(splitmix64(seed, item + 1), m + 1);
}

}  // namespace semd
