// Launch arguments of the Array-OL repetition with a linear integer
// elementary task on uint8 arrays (passed by value; pattern tables in device
// memory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aol {

constexpr int kLinRank = 4;
constexpr int kLinMaxIn = 1024;  // input pattern elements
constexpr int kLinMaxOut = 16;   // output pattern elements
constexpr int kLinThreads = 256;

struct LinearArgs {
  const uint8_t* in;
  uint8_t* out;
  int64_t nrep;                         // points of the repetition space
  int32_t rr;                           // repetition rank
  int32_t R[kLinRank];                  // repetition space (row-major; lanes run along the last dim)
  int32_t inc[kLinRank], oinc[kLinRank];  // (kLinThreads * paving along the last rep dim) mod S, per dim
  // input array and tiler
  int32_t ra;
  int32_t S[kLinRank], st[kLinRank];    // shape, strides (elements)
  int32_t o[kLinRank];                  // origin, reduced mod S
  int32_t P[kLinRank][kLinRank];        // paving [dim][rep dim], reduced mod S
  int32_t lo[kLinRank], hi[kLinRank];   // extent of the fitting offsets along each dim
  // output array and tiler
  int32_t ro;
  int32_t So[kLinRank], sto[kLinRank];
  int32_t oo[kLinRank];
  int32_t Po[kLinRank][kLinRank];
  int32_t olo[kLinRank], ohi[kLinRank];
  int32_t n_pairs;                      // input pattern elements, in pairs (an odd count is padded)
  int32_t n_out;                        // output pattern elements
  // Device table (int32), uniform reads:
  //   ioff[2 * n_pairs]            flat offset of input element i (pattern inside the array)
  //   ifd[ra][2 * n_pairs]         fitting offset of element i along each dim, reduced mod S
  //   wpair[n_pairs][NOUT]         weights of elements 2k and 2k+1 for output j, packed int16 pairs
  //   bias[NOUT]                   bias[j] + 128 (the rounding), then
  //   ooff[NOUT], ofd[ro][NOUT]    output pattern offsets as for the input
  const int32_t* tab;
  int32_t t_ifd, t_w, t_bias, t_ooff, t_ofd;  // offsets (int32 entries) of the table's parts
  // Point-by-point kernel, rows of at most kLinThreads points: thread t takes
  // point (t + rot) mod R[rr - 1] of its row (a bijection), so that the points
  // whose pattern crosses a border, a cyclic run along the row, share one
  // wave instead of diverging two. 0 otherwise.
  int32_t rot;
};

// Staged form: a workgroup takes C = kLinThreads * ppt consecutive points of
// one row of the repetition space (every index but the last fixed). Where
// consecutive points advance both arrays by constant flat strides P and Po,
// the input bytes the chunk's points read lie in a few contiguous ranges (one
// per group of pattern elements whose offsets are close): those are loaded
// into LDS with 16-byte loads, and the points read their pattern from there.
// Output elements grouped in runs of Po consecutive offsets cover their
// ranges densely: the points write into LDS and the workgroup stores whole
// 16-byte chunks. Points whose pattern crosses an array border (or whose
// coordinates wrap inside the chunk) take the point-by-point path. LDS holds
// first, per chunk, each element's position relative to a point's flat
// position (4 * (2 n_pairs + NOUT) bytes, rounded to 16), then the groups.
constexpr int kLinGroups = 4;          // input / output element groups at most
constexpr int kLinStageLds = 40 * 1024;  // LDS bytes of a staged workgroup at most
constexpr int kLinStageMaxIn = 32;       // input pattern elements of a staged plan at most
constexpr int64_t kLinCoordTable = 1 << 22;  // table entries (int32) of a staged plan at most

struct LinearStage {
  int32_t ppt;             // points per thread (0: staged form not used)
  int32_t chunks;          // workgroups per row
  int32_t P, Po;           // flat strides between consecutive points (input, output), > 0
  int32_t ng, ngo;         // input groups; dense output groups (0: outputs stored point by point)
  int32_t gb[kLinGroups];  // input group: least flat offset of its elements
  int32_t gs[kLinGroups];  // input group: extent of its offsets (largest - least + 1)
  int32_t gl[kLinGroups];  // input group: LDS byte base
  int32_t ob[kLinGroups];  // output group: least flat offset (its elements are ob .. ob + Po - 1)
  int32_t ol[kLinGroups];  // output group: LDS byte base
  int32_t lds_bytes;
  // table offsets: group of each input element (2 n_pairs), of each output
  // element (NOUT), and per group (kLinGroups) gb, gl, ob, ol
  int32_t t_eg, t_og, t_grp;
  int64_t n_in, n_out;     // elements of the input and output arrays
  // Per chunk (workgroup) g, at cq + 2 g: the flat input and output
  // positions of its first point, or -1 when the chunk is not clean (some
  // point's pattern crosses an array border, or a coordinate wraps between
  // the chunk's first and last point), computed on the host.
  int32_t cq;
  uint32_t mg_R[kLinRank];  // floor(2^32 / R[k]) + 1, and of chunks at [last]
};

hipError_t linear_launch(int nout, const LinearArgs& a, hipStream_t stream);
hipError_t linear_staged_launch(int nout, const LinearArgs& a, const LinearStage& st, hipStream_t stream);

}  // namespace aol
