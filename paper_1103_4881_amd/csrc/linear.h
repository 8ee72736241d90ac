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
};

hipError_t linear_launch(int nout, const LinearArgs& a, hipStream_t stream);

}  // namespace aol
