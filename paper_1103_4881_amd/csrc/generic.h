// Launch arguments of the generic weighted-sum repetition (passed by value).
#pragma once
#include <stdint.h>

namespace aol {

constexpr int kWsumMaxRank = 4;
constexpr int kMaxPat = 64;  // pattern elements

struct WsumArgs {
  const float* in;
  float* out;
  int32_t ra, rr, ro;                    // input array rank, repetition rank, output array rank
  int32_t S[kWsumMaxRank], st[kWsumMaxRank];  // input shape, strides (elements)
  int32_t R[kWsumMaxRank];               // repetition space
  int32_t o[kWsumMaxRank];               // input origin, reduced mod S
  int32_t P[kWsumMaxRank][kWsumMaxRank];  // input paving [dim][rep], reduced mod S
  int32_t P_loop[kWsumMaxRank];          // P[.][k_loop]
  int32_t lo[kWsumMaxRank], hi[kWsumMaxRank];  // extent of the fitting offsets along each dim
  int32_t npat;
  int32_t off[kMaxPat];                  // flat offset of each pattern element (pattern inside the array)
  int32_t fd[kWsumMaxRank][kMaxPat];     // fitting offset per dim, reduced mod S (border path)
  float w[kMaxPat];
  int32_t out_identity;                  // output tiler is B[r] row-major over the repetition space
  int32_t So[kWsumMaxRank], sto[kWsumMaxRank];  // output shape, strides
  int32_t oo[kWsumMaxRank];
  int32_t Po[kWsumMaxRank][kWsumMaxRank];
  int32_t Po_loop[kWsumMaxRank];
  int64_t ostr_rep[kWsumMaxRank];        // identity output: stride of each repetition dim
  int32_t k_lane, k_loop;                // repetition dims along lanes / along each thread's loop
  int32_t nb_lane, nb_loop;              // 64-wide blocks along k_lane / k_loop
  int32_t other[kWsumMaxRank];
  int32_t n_other;
  int32_t transpose;                     // stage results in LDS and store along k_loop
  // Staged form: the input box a 64x64 block of points reads (unwrapped
  // coordinates lo + [0, bn) per dim, lo = o + Ps.r_corner + dlo) is loaded
  // into LDS once; pattern element i of point (lane, jj) is then
  // box[lane*lstep + jj*jstep + offl[i]].
  int32_t use_box;
  int32_t Ps[kWsumMaxRank][kWsumMaxRank];  // paving, signed representative nearest zero
  int32_t dlo[kWsumMaxRank];             // box origin relative to the block's corner point
  int32_t bn[kWsumMaxRank];              // box extent per dim
  int32_t box_rows;                      // product of the extents of all but the last dim
  int32_t box_elems;
  int32_t lstep, jstep;                  // box offset per lane / per loop point
  int32_t offl[kMaxPat];                 // box offset of each pattern element (dlo folded in)
};

constexpr int kWsumBoxMaxBytes = 48 * 1024;  // box in LDS per workgroup
constexpr int kWsumBoxPoints = 8;            // staged form: points per thread along the loop dimension

}  // namespace aol
