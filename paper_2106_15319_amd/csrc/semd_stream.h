// Streaming (multi-workgroup) Serial-EMD path: per-signal state and the
// launchers of its kernels (semd_stream.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace semd {

// Samples per tile (one workgroup of a tile kernel).
constexpr int kTile = 2048;

// What the scan needs from, and gives back to, one tile.
struct TileInfo {
  int32_t cnt[2];     // extrema found by detect, continuation run excluded
  int32_t tot[2];     // extrema of the tile, continuation run resolved
  int32_t off[2];     // rank of the tile's first knot of each kind
  int32_t lastkey;    // 4*index + step kind of the tile's last run start, -1 if none
  int32_t carry;      // key of the run holding the tile's first sample
  int32_t cont;       // that run started before the tile
  int32_t cont_exit;  // direction the run is left in inside the tile, 0 if not
  int32_t bad;        // the tile holds NaN/Inf input
  int32_t pad;
};

// Dynamic state of one signal.
struct SigStatus {
  int32_t active;   // the decomposition goes on
  int32_t skip;     // the current IMF's remaining sifts are skipped
  int32_t nimf;     // IMFs written
  int32_t bad;      // input holds NaN/Inf
  int32_t n[2];     // maxima / minima of the current sift
  int64_t n_sifts;  // sifts performed
  int64_t n_knots;  // knots used, mirrored ones included
};

// One signal of a streaming batch.
struct StreamSig {
  const double* X;
  double* out;
  int32_t* n_imfs;
  int64_t* stats;
  int64_t M, N;
  int32_t D, L;
  double beta;
  uint64_t key;
  int32_t flags;    // bit 0: add beta * noise
  int32_t ntiles;
  double* h;        // candidate, L doubles
  double* r;        // residue, L doubles
  int32_t* kt[2];   // knot abscissae (maxima, minima), cap each
  double* ky[2];    // knot values
  double* km[2];    // second derivatives
  int32_t cap;      // knots per envelope
  int32_t pad;
  TileInfo* tinfo;  // ntiles
  SigStatus* st;
};

hipError_t st_init(const StreamSig* sigs, int n, hipStream_t s);
hipError_t st_load(const StreamSig* sigs, const int2* tiles, int ntiles, hipStream_t s);
// One sift (detect, scan, compact, solve, eval) of every running signal; s is
// the sift's index within its IMF.
hipError_t st_sift(const StreamSig* sigs, int nsig, const int2* tiles, int ntiles,
                   const int4* blocks, int nblocks, int s, hipStream_t st);
hipError_t st_imf_end(const StreamSig* sigs, int nsig, const int2* tiles, int ntiles,
                      hipStream_t s);
hipError_t st_final(const StreamSig* sigs, const int2* tiles, int ntiles, int K,
                    hipStream_t s);
// Solve blocks one envelope of `cap` knots needs.
int stream_solve_blocks(int cap);

}  // namespace semd
