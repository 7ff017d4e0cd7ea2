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

#include "semd_device.h"

namespace semd {
namespace {

using namespace dev;

constexpr int kAggBytes = 256;

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
      detect_extrema<NT, C>(h, 0, L, L, tid, 0, 0.0, pub_first, pub_last, pub_key, carry,
                            maxbits, minbits, cmax, cmin, nullptr, nullptr);
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
        emit_knots<C>(h, maxbits, carry, base, nv, L, emax, nmax, kt, ky, nkmax);
        emit_knots<C>(h, minbits, carry, base, nv, L, emin, nmin, kt + nkmax, ky + nkmax,
                      nkmin);
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
        emit_knots<C>(h, maxbits, carry, base, nv, L, emax, nmax, kt, ky, nkmax);
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
        emit_knots<C>(h, minbits, carry, base, nv, L, emin, nmin, kt, ky, nkmin);
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
  detect_extrema<NT, C>(h, 0, L, L, tid, 0, 0.0, pub_first, pub_last, pub_key, carry, maxbits,
                        minbits, cmax, cmin, nullptr, nullptr);
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
