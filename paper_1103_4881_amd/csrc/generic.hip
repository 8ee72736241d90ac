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
//
// Staged form (BOX): when the input elements a block of points reads lie in a
// box small enough for LDS, the workgroup first loads that box (rows along
// the input's contiguous axis, the modulo wrap applied while loading), then
// every pattern element of every point is an LDS read at a constant offset
// from the point's base; each input element comes from HBM once per block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generic.h"

namespace aol {

// The arrays are read and written through global address-space pointers:
// pointers taken from a by-value argument structure are generic to the
// compiler, and generic accesses become flat instructions.
typedef const __attribute__((address_space(1))) float* gin_t;
typedef __attribute__((address_space(1))) float* gout_t;

// Weighted sum of one pattern: the gathers are issued 8 at a time, so that
// several are in flight instead of one load waiting for the previous one.
template <class Off>
__device__ __forceinline__ float wsum_pattern(const WsumArgs& a, Off off) {
  gin_t in = (gin_t)a.in;
  float acc = 0.f;
  int i = 0;
  for (; i + 8 <= a.npat; i += 8) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = in[off(i + k)];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc = __builtin_fmaf(a.w[i + k], v[k], acc);
  }
  for (; i < a.npat; ++i) acc = __builtin_fmaf(a.w[i], in[off(i)], acc);
  return acc;
}

// Staged form: the weighted sums of this thread's PT points from the box,
// pattern element outermost so that the points' LDS reads are independent
// (PT in flight per element, few registers).
template <int PT>
__device__ __forceinline__ void wsum_box_points(const WsumArgs& a, const float* pb0, int jstep, float (&acc)[PT]) {
#pragma unroll
  for (int j = 0; j < PT; ++j) acc[j] = 0.f;
  // four pattern elements per iteration: their offsets and weights come in one
  // batch of scalar loads, and 4*PT box reads are in flight
#pragma unroll 4
  for (int i = 0; i < a.npat; ++i) {
    const float* p = pb0 + a.offl[i];
    const float w = a.w[i];
#pragma unroll
    for (int j = 0; j < PT; ++j) acc[j] = __builtin_fmaf(w, p[j * jstep], acc[j]);
  }
}

// PT: points per thread along the loop dimension (a block is 64 x 4*PT
// points): 16 for the direct form, 8 for the staged form (a smaller box, so
// more workgroups per compute unit overlap their loads with others' sums).
template <bool BOX>
__global__ __launch_bounds__(256) void k_wsum(WsumArgs a) {
  constexpr int PT = BOX ? 8 : 16;
  constexpr int BJ = 4 * PT;  // block extent along the loop dimension
  __shared__ float tile[64][BJ + 1];
  extern __shared__ float box[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // block -> (lane block, loop block, other repetition indices), uniform and
  // in 32 bits (fewer than 2^31 blocks); arrays indexed by unrolled
  // constants only, so they stay in scalar registers
  uint32_t blk = blockIdx.x;
  const int bl = (int)(blk % (uint32_t)a.nb_lane);
  blk /= (uint32_t)a.nb_lane;
  const int bp = (int)(blk % (uint32_t)a.nb_loop);
  blk /= (uint32_t)a.nb_loop;
  int rc[kWsumMaxRank];  // the block's corner point
#pragma unroll
  for (int k = kWsumMaxRank - 1; k >= 0; --k) {
    rc[k] = 0;
    if (k < a.rr && k != a.k_lane && k != a.k_loop) {
      rc[k] = (int)(blk % (uint32_t)a.R[k]);
      blk /= (uint32_t)a.R[k];
    } else if (k == a.k_lane) {
      rc[k] = bl * 64;
    } else if (k == a.k_loop) {
      rc[k] = bp * BJ;
    }
  }
  const int r_lane = bl * 64 + lane;
  const int r_loop0 = bp * BJ + wave * PT;
  int64_t r[kWsumMaxRank];  // this thread's first point
#pragma unroll
  for (int k = 0; k < kWsumMaxRank; ++k)
    r[k] = rc[k] + (k == a.k_lane ? lane : 0) + (k == a.k_loop ? wave * PT : 0);
  const bool lane_ok = r_lane < a.R[a.k_lane];

  // wrapped base index of the first point of this thread, input (direct
  // form only) and output (a non-identity output tiler only)
  int base[kWsumMaxRank], obase[kWsumMaxRank];
  int64_t oflat = 0;
#pragma unroll
  for (int d = 0; d < kWsumMaxRank; ++d) {
    base[d] = 0;
    obase[d] = 0;
    if (!BOX && d < a.ra) {
      int64_t v = a.o[d];
      for (int k = 0; k < a.rr; ++k) v += (int64_t)a.P[d][k] * r[k];
      base[d] = (int)(v % a.S[d]);
    }
    if (!a.out_identity && d < a.ro) {
      int64_t v = a.oo[d];
      for (int k = 0; k < a.rr; ++k) v += (int64_t)a.Po[d][k] * r[k];
      obase[d] = (int)(v % a.So[d]);
    }
  }
  if (a.out_identity) {
    for (int k = 0; k < a.rr; ++k) oflat += r[k] * a.ostr_rep[k];
  }

  if constexpr (BOX) {
    // box origin of the block (its corner point: lane 0, loop point 0), wrapped
    int lo[kWsumMaxRank];
#pragma unroll
    for (int d = 0; d < kWsumMaxRank; ++d) {
      lo[d] = 0;
      if (d < a.ra) {
        int64_t v = (int64_t)a.o[d] + a.dlo[d];
#pragma unroll
        for (int k = 0; k < kWsumMaxRank; ++k) v += (int64_t)a.Ps[d][k] * rc[k];
        v %= a.S[d];
        lo[d] = (int)(v < 0 ? v + a.S[d] : v);
      }
    }
    const int last = a.ra - 1;
    const int rowlen = a.bn[last];
    // the input is under 4 GiB in this form: a uniform base plus a 32-bit byte offset per element
    const __attribute__((address_space(1))) uint8_t* inb = (const __attribute__((address_space(1))) uint8_t*)a.in;
    auto ld = [&](uint32_t elem) { return *(gin_t)(inb + (uint64_t)(elem * 4u)); };
    // rows along the contiguous axis, eight rows per wave and iteration with
    // every load issued before the first store (up to 32 loads per lane in
    // flight).
    // The wrapped columns of the lane's elements are the same in every row:
    // computed once. Row coordinates advance by a counter with carries.
    const int nt = (rowlen + 63) / 64;  // 64-element pieces of a row
    auto wrap_col = [&](int piece) {  // wrapped column of the lane's element of a 64-element piece
      int c = lo[last] + min(piece * 64 + lane, rowlen - 1);
      if (c >= a.S[last]) c -= a.S[last];
      if (c >= a.S[last]) c -= a.S[last];
      return c;
    };
    int col[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) col[k] = wrap_col(k);
    int t[kWsumMaxRank] = {0, 0, 0, 0};  // coordinates of row `row` in the box (all dims but the last)
    auto advance = [&](int by) {
      for (int d = last - 1; d >= 0 && by > 0; --d) {
        const int v = t[d] + by;
        by = v / a.bn[d];
        t[d] = v - by * a.bn[d];
      }
    };
    constexpr int QR = 8;  // rows per wave and iteration
    advance(wave * QR);
    for (int row0 = wave * QR; row0 < a.box_rows; row0 += 4 * QR) {
      int g[QR];
      int tq[kWsumMaxRank] = {t[0], t[1], t[2], t[3]};
#pragma unroll
      for (int q = 0; q < QR; ++q) {
        int gg = 0;
#pragma unroll
        for (int d = 0; d < kWsumMaxRank - 1; ++d) {
          if (d >= last) break;
          int c = lo[d] + tq[d];  // lo < S and t < extent <= 2S: two subtractions wrap it
          if (c >= a.S[d]) c -= a.S[d];
          if (c >= a.S[d]) c -= a.S[d];
          gg += c * a.st[d];
        }
        g[q] = gg;
        // next row (past the last row: stays in the box, loaded and not stored)
#pragma unroll
        for (int d = kWsumMaxRank - 2; d >= 0; --d) {
          if (d >= last) continue;
          if (++tq[d] < a.bn[d]) break;
          tq[d] = 0;
        }
      }
      for (int t0 = 0; t0 < nt; t0 += 4) {
        float v[QR][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k > 0 && t0 + k >= nt) break;  // uniform
          const int c = t0 == 0 ? col[k] : wrap_col(t0 + k);
#pragma unroll
          for (int q = 0; q < QR; ++q) v[q][k] = ld((uint32_t)(g[q] + c));
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k > 0 && t0 + k >= nt) break;
          const int tt = (t0 + k) * 64 + lane;
          // an element past the row or past the last row goes to the lane's slot after the box
          const int dst0 = tt < rowlen ? row0 * rowlen + tt : a.box_elems + lane;
#pragma unroll
          for (int q = 0; q < QR; ++q) box[row0 + q < a.box_rows && tt < rowlen ? dst0 + q * rowlen : a.box_elems + lane] = v[q][k];
        }
      }
      advance(4 * QR);
    }
    __syncthreads();
  }
  float bacc[BOX ? PT : 1];
  if constexpr (BOX) wsum_box_points<PT>(a, box + lane * a.lstep + wave * PT * a.jstep, a.jstep, bacc);

#pragma unroll(BOX ? PT : 1)
  for (int j = 0; j < PT; ++j) {
    const int rl = r_loop0 + j;
    const bool ok = lane_ok && rl < a.R[a.k_loop];
    float acc = 0.f;
    if constexpr (BOX) {
      acc = bacc[BOX ? j : 0];  // points outside the repetition space read inside the box all the same
    } else if (ok) {
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
        acc = wsum_pattern(a, [&](int i) { return flat + a.off[i]; });
      } else {
        acc = wsum_pattern(a, [&](int i) {
          int f = 0;
#pragma unroll
          for (int d = 0; d < kWsumMaxRank; ++d) {
            if (d < a.ra) {
              uint32_t v = (uint32_t)base[d] + (uint32_t)a.fd[d][i];  // both in [0, S): no wrap past 2^32
              if (v >= (uint32_t)a.S[d]) v -= (uint32_t)a.S[d];
              f += (int)v * a.st[d];
            }
          }
          return f;
        });
      }
    }
    if (a.transpose) {
      tile[lane][wave * PT + j] = acc;
    } else if (ok) {
      int64_t of = oflat;
      if (!a.out_identity) {
        of = 0;
#pragma unroll
        for (int d = 0; d < kWsumMaxRank; ++d)
          if (d < a.ro) of += (int64_t)obase[d] * a.sto[d];
      }
      ((gout_t)a.out)[of] = acc;
    }
    // next point along the loop dimension
#pragma unroll
    for (int d = 0; d < kWsumMaxRank; ++d) {
      if (!BOX && d < a.ra) {
        uint32_t v = (uint32_t)base[d] + (uint32_t)a.P_loop[d];
        if (v >= (uint32_t)a.S[d]) v -= (uint32_t)a.S[d];
        base[d] = (int)v;
      }
      if (!a.out_identity && d < a.ro) {
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
    const int rl = bp * BJ + lane;
    for (int row = wave; row < 64; row += 4) {
      const int rla = bl * 64 + row;
      if (lane < BJ && rla < a.R[a.k_lane] && rl < a.R[a.k_loop])
        ((gout_t)a.out)[rowbase + (int64_t)rla * a.ostr_rep[a.k_lane] + (int64_t)rl * a.ostr_rep[a.k_loop]] = tile[row][lane];
    }
  }
}

using WsumFn = void (*)(WsumArgs);

static WsumFn wsum_pick(const WsumArgs& a) { return a.use_box ? k_wsum<true> : k_wsum<false>; }

hipError_t wsum_prepare() {
  return hipFuncSetAttribute((const void*)k_wsum<true>, hipFuncAttributeMaxDynamicSharedMemorySize, kWsumBoxMaxBytes + 256);
}

hipError_t wsum_launch(const WsumArgs& a, int64_t blocks, hipStream_t stream) {
  const size_t lds = a.use_box ? (size_t)(a.box_elems + 64) * 4 : 0;  // and one spill slot per lane
  hipLaunchKernelGGL(wsum_pick(a), dim3((unsigned)blocks), dim3(256), lds, stream, a);
  return hipGetLastError();
}

}  // namespace aol
