// Streaming (multi-workgroup) Serial-EMD path: per-signal state and the
// launchers of its kernels (semd_stream.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace semd {

// Samples per tile (one workgroup of a tile kernel) and threads per tile.
constexpr int kTile = 2048;
constexpr int kTileThreads = 256;
// Knots of one kind a tile can hold (a strict extremum needs two steps).
constexpr int kTileKnots = kTile / 2 + 8;

// What the scan needs from, and gives back to, one tile.
struct TileInfo {
  int32_t cnt[2];     // extrema found by detection, the continued run excluded
  int32_t tot[2];     // extrema of the tile, the continued run resolved
  int32_t off[2];     // rank of the tile's first knot of each kind
  int32_t lastkey;    // 4*index + step kind of the tile's last run start, -1 if none
  int32_t carry;      // key of the run holding the tile's first sample
  int32_t cont;       // that run started before the tile
  int32_t cont_exit;  // direction the run is left in inside the tile, 0 if not
  int32_t bad;        // the tile holds NaN/Inf input
  int32_t cont_pos;   // sample where that run ends (its extremum's sample), -1 if none
  int32_t cont_knot;  // bit e: the continued run is an extremum of kind e (scan)
  int32_t pad;
  double cont_y;      // the continued run's value
  double sd_num;      // sums over the tile's samples of a sift step: m^2
  double sd_den;      //   and h^2 of the candidate before the sift
};

// What a step does to a signal (decided by the scan from the current
// candidate's extrema).
enum StepAction : int32_t {
  kIdle = 0,      // finished: nothing
  kSift = 1,      // one sift
  kSiftLast = 2,  // one sift, then the IMF ends
  kEndImf = 3,    // the candidate is not siftable, or the last sift met the SD
                  // criterion: the IMF ends without a sift
  kFinish = 4     // the residue is not siftable (or the input is bad): outputs final
};

// Dynamic state of one signal.
struct SigStatus {
  int32_t active;   // final outputs not written yet
  int32_t sift;     // sifts done in the current IMF
  int32_t nimf;     // IMFs ended
  int32_t bad;      // input holds NaN/Inf
  int32_t action;   // this step's StepAction
  int32_t slot;     // output slot of the IMF ending this step
  int32_t fin;      // this step writes the final outputs
  int32_t done;     // final outputs written
  int32_t n[2];     // maxima / minima of the current sift
  int32_t tr_rec;   // trace entry of this step's detection record, -1 if none
  int32_t tr_n[2];  //   and its maxima / minima counts
  int32_t in_r;     // this step's candidate is in r, not h (set by the scan)
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
  int64_t slot_stride;  // doubles from one output slot to the next
  double sd;        // SD stopping threshold; 0: fixed sift count
  const double* addend;  // added (scaled) under kAddBuffer
  const double* scale;   // beta on the device under kScaleOnDevice
  int32_t flags;    // as a WorkItem's
  int32_t ntiles;
  int32_t K;        // max IMFs
  int32_t S;        // sifts per IMF
  double* h;        // candidate, L doubles
  double* r;        // residue, L doubles
  int32_t* kt[2];   // knot abscissae (maxima, minima), cap each
  double* ky[2];    // knot values
  double* km[2];    // the envelopes' second derivatives at the knots
  int32_t cap;      // knots per envelope
  int32_t pad;
  TileInfo* tinfo;  // ntiles
  double* edge;     // ntiles x 2: a tile's first and last sample before the sift,
                    // then ntiles x 2: the same of the residue before an IMF-ending sift
  int32_t* trank;   // ntiles x kTileThreads: knots of each kind the tile's earlier
                    // threads hold (ranks within the tile; maxima in the low 16 bits,
                    // minima in the high 16)
  int32_t* lpos[2]; // ntiles x kTileKnots: the tile's knots at tile-local ranks
  double* lval[2];  //   (positions and values), written by detection
  SigStatus* st;
  int32_t* trace;   // extremum decisions (layout of launch_resident_trace), or nullptr
  int32_t trace_cap;
  int32_t pad2;
};

// r = serialized input (+ noise), the first candidate (read from r by the
// first step), its extrema detected, and a fresh status, for the signals
// whose tiles are listed.
hipError_t st_load(const StreamSig* sigs, const int2* tiles, int ntiles, hipStream_t s);
// One step of every listed signal: scan (decides the step's action), compact
// and solve (sifting signals), eval (sift, IMF end, final outputs, and the
// next candidate's extrema).
// sd: some signal uses the SD stopping rule (its sums are accumulated).
// trace: also record each detection of the signals that carry a trace.
// marks (5 events, or nullptr): recorded before the step and after each of
// its scan, compact, solve and eval launches, for kernel timing.
hipError_t st_step(const StreamSig* sigs, int nsig, const int2* tiles, int ntiles,
                   const int4* blocks, int nblocks, hipStream_t s, bool sd, bool trace = false,
                   const hipEvent_t* marks = nullptr);
// The descriptor of the one signal g and its tile and solve-block tables
// (g.ntiles entries, and two per solve workgroup: stream_solve_groups(g.cap,
// stream_solve_fold(2 * stream_solve_blocks(g.cap))) each), written on the
// device from a kernel argument: no host staging buffer, no allocation.
hipError_t st_put_single(const StreamSig& g, StreamSig* dsig, int2* tiles, int4* blocks,
                         hipStream_t s);
// done[i] = status of signal i has its final outputs written.
hipError_t st_gather_done(const StreamSig* sigs, int nsig, int32_t* done, hipStream_t s);
// Solve blocks one envelope of `cap` knots spans (an upper bound on the
// solve-table entries it takes).
int stream_solve_blocks(int cap);
// The fold of a launch whose envelopes span `total_blocks` solve blocks, and
// the workgroups (solve-table entries) one envelope of `cap` knots takes
// under it: workgroup z of G handles blocks z, z + G, ...  The fold gives
// one workgroup slot per `target` blocks (a tuned value; 0 takes the
// built-in one), at most the compiled maximum.
int stream_solve_fold(int64_t total_blocks, int target = 0);
int stream_solve_groups(int cap, int fold);

}  // namespace semd
