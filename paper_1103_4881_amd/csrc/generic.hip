// General Array-OL repetition with a weighted-sum elementary task (float32).
//
// Sec. III-A and its tiler footnote: a repetitive task runs one elementary
// task per point r of its repetition space; the input tiler gathers pattern
// element i from A[(o + P.r + F.i) mod S], and an output tiler writes the
// single result to B[(o' + P'.r) mod S']. Here the elementary task is
// y = sum_i w[i] * pattern[i].
//
// Work mapping: a workgroup covers a 64 x 64 block of two repetition
// dimensions with every other repetition index fixed. Lanes run along the
// dimension whose paving column walks the input's contiguous axis (the
// gathers of one pattern element are then adjacent addresses); each thread
// walks 16 points of the second dimension, updating the wrapped base index
// incrementally. A pattern that stays inside the array uses constant flat
// offsets; one that crosses a border wraps each axis separately. When the
// output's contiguous dimension is the per-thread one, results go through a
// transposed LDS tile so that stores are contiguous too.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generic.h"

namespace aol {

__global__ __launch_bounds__(256) void k_wsum(WsumArgs a) {
  __shared__ float tile[64][65];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // block -> (lane block, loop block, other repetition indices)
  int64_t blk = blockIdx.x;
  const int bl = (int)(blk % a.nb_lane);
  blk /= a.nb_lane;
  const int bp = (int)(blk % a.nb_loop);
  blk /= a.nb_loop;
  int64_t r[kWsumMaxRank];
#pragma unroll
  for (int k = 0; k < kWsumMaxRank; ++k) r[k] = 0;
  for (int j = a.n_other - 1; j >= 0; --j) {
    const int k = a.other[j];
    r[k] = blk % a.R[k];
    blk /= a.R[k];
  }
  const int r_lane = bl * 64 + lane;
  const int r_loop0 = bp * 64 + wave * 16;
  r[a.k_lane] = r_lane;
  r[a.k_loop] = r_loop0;
  const bool lane_ok = r_lane < a.R[a.k_lane];

  // wrapped base index of the first point of this thread, input and output
  int base[kWsumMaxRank], obase[kWsumMaxRank];
  int64_t oflat = 0;
#pragma unroll
  for (int d = 0; d < kWsumMaxRank; ++d) {
    base[d] = 0;
    obase[d] = 0;
    if (d < a.ra) {
      int64_t v = a.o[d];
      for (int k = 0; k < a.rr; ++k) v += (int64_t)a.P[d][k] * r[k];
      base[d] = (int)(v % a.S[d]);
    }
    if (d < a.ro) {
      int64_t v = a.oo[d];
      for (int k = 0; k < a.rr; ++k) v += (int64_t)a.Po[d][k] * r[k];
      obase[d] = (int)(v % a.So[d]);
    }
  }
  if (a.out_identity) {
    for (int k = 0; k < a.rr; ++k) oflat += r[k] * a.ostr_rep[k];
  }

  for (int j = 0; j < 16; ++j) {
    const int rl = r_loop0 + j;
    const bool ok = lane_ok && rl < a.R[a.k_loop];
    float acc = 0.f;
    if (ok) {
      bool inside = true;
      int flat = 0;
#pragma unroll
      for (int d = 0; d < kWsumMaxRank; ++d) {
        if (d < a.ra) {
          inside = inside && (base[d] >= -a.lo[d]) && (base[d] < a.S[d] - a.hi[d]);
          flat += base[d] * a.st[d];
        }
      }
      if (inside) {
        const float* p = a.in + flat;
        for (int i = 0; i < a.npat; ++i) acc = __builtin_fmaf(a.w[i], p[a.off[i]], acc);
      } else {
        for (int i = 0; i < a.npat; ++i) {
          int f = 0;
#pragma unroll
          for (int d = 0; d < kWsumMaxRank; ++d) {
            if (d < a.ra) {
              uint32_t v = (uint32_t)base[d] + (uint32_t)a.fd[d][i];  // both in [0, S): no wrap past 2^32
              if (v >= (uint32_t)a.S[d]) v -= (uint32_t)a.S[d];
              f += (int)v * a.st[d];
            }
          }
          acc = __builtin_fmaf(a.w[i], a.in[f], acc);
        }
      }
    }
    if (a.transpose) {
      tile[lane][wave * 16 + j] = acc;
    } else if (ok) {
      int64_t of = oflat;
      if (!a.out_identity) {
        of = 0;
#pragma unroll
        for (int d = 0; d < kWsumMaxRank; ++d)
          if (d < a.ro) of += (int64_t)obase[d] * a.sto[d];
      }
      a.out[of] = acc;
    }
    // next point along the loop dimension
#pragma unroll
    for (int d = 0; d < kWsumMaxRank; ++d) {
      if (d < a.ra) {
        uint32_t v = (uint32_t)base[d] + (uint32_t)a.P_loop[d];
        if (v >= (uint32_t)a.S[d]) v -= (uint32_t)a.S[d];
        base[d] = (int)v;
      }
      if (d < a.ro) {
        uint32_t v = (uint32_t)obase[d] + (uint32_t)a.Po_loop[d];
        if (v >= (uint32_t)a.So[d]) v -= (uint32_t)a.So[d];
        obase[d] = (int)v;
      }
    }
    oflat += a.ostr_rep[a.k_loop];
  }

  if (a.transpose) {
    // identity output whose contiguous dimension is the loop dimension:
    // lanes now run along it
    __syncthreads();
    int64_t rowbase = 0;
    for (int k = 0; k < a.rr; ++k)
      if (k != a.k_lane && k != a.k_loop) rowbase += r[k] * a.ostr_rep[k];
    const int rl = bp * 64 + lane;
    for (int row = wave; row < 64; row += 4) {
      const int rla = bl * 64 + row;
      if (rla < a.R[a.k_lane] && rl < a.R[a.k_loop])
        a.out[rowbase + (int64_t)rla * a.ostr_rep[a.k_lane] + (int64_t)rl * a.ostr_rep[a.k_loop]] = tile[row][lane];
    }
  }
}

hipError_t wsum_launch(const WsumArgs& a, int64_t blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k_wsum, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace aol
