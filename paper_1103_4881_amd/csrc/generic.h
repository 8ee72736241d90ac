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
  uint32_t mg_lane, mg_loop, mg_R[kWsumMaxRank];  // floor(2^32 / divisor) + 1 of nb_lane, nb_loop, R
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
  // Box origins without 64-bit arithmetic on the device: lo[d] = (c0[d] +
  // sum_k ctab[ctab_off[k] + b_k * ra + d]) mod S[d], b_k the block's index
  // along repetition dim k (every term already reduced mod S[d]); NULL: the
  // origin is computed directly.
  const int32_t* ctab;
  int32_t ctab_off[kWsumMaxRank];
  int32_t c0[kWsumMaxRank];
  // Staged form, values shared along the loop dimension: pattern elements
  // whose box offsets differ by a multiple of jstep read, at neighbouring
  // points, the same box elements. Class c (ncls of them) lists its offset
  // key and first multiple mmin, then em weights (float bits) for the
  // multiples mmin .. mmin + em - 1 (zero where no element sits): point j
  // adds sum_e w[e] * box[base + key + (mmin + e + j) * jstep]. NULL: one
  // read per pattern element and point.
  const int32_t* cls;
  int32_t ncls, em;
  int32_t ctab_cls;  // host: offset of the class table inside the device table
};

constexpr int kWsumClassWidths[] = {3, 5, 8};  // kernel instances by the widest class

constexpr int kWsumBoxMaxBytes = 48 * 1024;  // box in LDS per workgroup
constexpr int kWsumBoxPoints = 8;            // staged form: points per thread along the loop dimension

}  // namespace aol
