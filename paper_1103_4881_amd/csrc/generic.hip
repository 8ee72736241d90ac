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
// the input's contiguous axis, the modulo wrap applied while loading; the
// rows' wrapped offsets computed by the lanes in parallel, the box origin
// from a host table of per-block terms), then every pattern element of
// every point is an LDS read at a constant offset from the point's base;
// each input element comes from HBM once per block. Pattern elements whose
// offsets differ by a multiple of the loop dimension's step read, at
// neighbouring points of a thread, the same box elements: such a class is
// read once per thread (PT + width - 1 reads) and weighted as a sliding
// window.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generic.h"

namespace aol {

// The arrays are read and written through global address-space pointers:
// pointers taken from a by-value argument structure are generic to the
// compiler, and generic accesses become flat instructions.
typedef const __attribute__((address_space(1))) float* gin_t;
#define AOL_WCONST __attribute__((address_space(4)))
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

// floor(n / d) for n, d < 2^31 from m = floor(2^32 / d) + 1: the product's
// high word is the quotient or one more, corrected by one comparison.
__device__ __forceinline__ uint32_t wsum_div(uint32_t n, uint32_t d, uint32_t m) {
  if (d == 1) return n;  // m would be 2^32 + 1
  uint32_t q = __umulhi(n, m);
  return q * d > n ? q - 1 : q;
}

// Staged form with reads shared along the loop dimension: per class, the
// box values of its multiples at the thread's PT points (PT + width - 1
// reads, the rest zero), then each multiple's weight times a sliding window
// of them.
template <int PT, int EM>
__device__ __forceinline__ void wsum_box_classes(const WsumArgs& a, const float* pb0, float (&acc)[PT]) {
  const AOL_WCONST int32_t* ct = (const AOL_WCONST int32_t*)a.cls;
#pragma unroll
  for (int j = 0; j < PT; ++j) acc[j] = 0.f;
  for (int c = 0; c < a.ncls; ++c) {
    const AOL_WCONST int32_t* e = ct + c * (2 + EM);
    const float* p = pb0 + e[0];  // the class's first multiple: key + mmin * jstep
    float w[EM];
    int nv = PT;  // values the class reads: PT + (its widest nonzero multiple)
#pragma unroll
    for (int m = 0; m < EM; ++m) {
      w[m] = __int_as_float(e[2 + m]);
      if (e[2 + m] != 0) nv = PT + m;
    }
    float v[PT + EM - 1];
#pragma unroll
    for (int t = 0; t < PT + EM - 1; ++t) v[t] = t < nv ? p[t * a.jstep] : 0.f;  // uniform bound
#pragma unroll
    for (int m = 0; m < EM; ++m)
#pragma unroll
      for (int j = 0; j < PT; ++j) acc[j] = __builtin_fmaf(w[m], v[j + m], acc[j]);
  }
}

// PT: points per thread along the loop dimension (a block is 64 x 4*PT
// points): 16 for the direct form, 8 for the staged form (a smaller box, so
// more workgroups per compute unit overlap their loads with others' sums).
// EM: the widest class of shared reads (0: one read per pattern element).
template <bool BOX, int EM>
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
  uint32_t q = wsum_div(blk, (uint32_t)a.nb_lane, a.mg_lane);
  const int bl = (int)(blk - q * (uint32_t)a.nb_lane);
  blk = q;
  q = wsum_div(blk, (uint32_t)a.nb_loop, a.mg_loop);
  const int bp = (int)(blk - q * (uint32_t)a.nb_loop);
  blk = q;
  int rc[kWsumMaxRank];  // the block's corner point
#pragma unroll
  for (int k = kWsumMaxRank - 1; k >= 0; --k) {
    rc[k] = 0;
    if (k < a.rr && k != a.k_lane && k != a.k_loop) {
      q = wsum_div(blk, (uint32_t)a.R[k], a.mg_R[k]);
      rc[k] = (int)(blk - q * (uint32_t)a.R[k]);
      blk = q;
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
    if (a.ctab) {
      // sum of terms each reduced mod S on the host: a few subtractions wrap it
      const AOL_WCONST int32_t* ct = (const AOL_WCONST int32_t*)a.ctab;
      int bk[kWsumMaxRank];
#pragma unroll
      for (int k = 0; k < kWsumMaxRank; ++k) bk[k] = k == a.k_lane ? bl : k == a.k_loop ? bp : rc[k];
#pragma unroll
      for (int d = 0; d < kWsumMaxRank; ++d) {
        lo[d] = 0;
        if (d < a.ra) {
          int v = a.c0[d];
#pragma unroll
          for (int k = 0; k < kWsumMaxRank; ++k) {
            if (k < a.rr) {
              v += ct[a.ctab_off[k] + bk[k] * a.ra + d];
              if (v >= a.S[d]) v -= a.S[d];
            }
          }
          lo[d] = v;
        }
      }
    } else {
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
    // Global offset of every box row (all dims but the last, the one before
    // the last fastest), wrapped per dim: one row per thread, into LDS
    // after the box and the spill slots.
    int* roff = reinterpret_cast<int*>(box + a.box_elems + 64);
    for (int q = threadIdx.x; q < a.box_rows; q += 256) {
      int rem = q, gg = 0;
#pragma unroll
      for (int d = kWsumMaxRank - 2; d >= 0; --d) {
        if (d >= last) continue;
        const int td = rem % a.bn[d];
        rem /= a.bn[d];
        int c = lo[d] + td;  // lo < S and td < extent <= 2S: two subtractions wrap it
        if (c >= a.S[d]) c -= a.S[d];
        if (c >= a.S[d]) c -= a.S[d];
        gg += c * a.st[d];
      }
      roff[q] = gg;
    }
    __syncthreads();
    constexpr int QR = 8;  // rows per wave and iteration
    for (int row0 = wave * QR; row0 < a.box_rows; row0 += 4 * QR) {
      int g[QR];
#pragma unroll
      for (int q = 0; q < QR; ++q) g[q] = roff[min(row0 + q, a.box_rows - 1)];  // past the last row: loaded, not stored
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
    }
    __syncthreads();
  }
  float bacc[BOX ? PT : 1];
  if constexpr (BOX && EM > 0) wsum_box_classes<PT, EM>(a, box + lane * a.lstep + wave * PT * a.jstep, bacc);
  else if constexpr (BOX) wsum_box_points<PT>(a, box + lane * a.lstep + wave * PT * a.jstep, a.jstep, bacc);

  if constexpr (BOX) {
    if (a.transpose) {  // the usual staged case: results go through the transposed tile
#pragma unroll
      for (int j = 0; j < PT; ++j) tile[lane][wave * PT + j] = bacc[j];
    }
  }
#pragma unroll(BOX ? PT : 1)
  for (int j = 0; j < PT; ++j) {
    if (BOX && a.transpose) break;  // uniform: stored above
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
    // output arrays hold fewer than 2^31 elements: 32-bit offsets
    uint32_t rowbase = 0;
    for (int k = 0; k < a.rr; ++k)
      if (k != a.k_lane && k != a.k_loop) rowbase += (uint32_t)r[k] * (uint32_t)a.ostr_rep[k];
    // A row of the tile is BJ points: with BJ = 32 the two halves of a wave
    // take rows r and r + 32 (33 * 32 = 32 mod 64 banks apart: no conflict).
    constexpr int HALVES = 64 / BJ;
    const int col = lane % BJ, half = lane / BJ;
    const int rl = bp * BJ + col;
    const uint32_t sl = (uint32_t)a.ostr_rep[a.k_lane];
    const int row0 = wave + half * 32;
    uint32_t of = rowbase + (uint32_t)(bl * 64 + row0) * sl + (uint32_t)rl * (uint32_t)a.ostr_rep[a.k_loop];
    const bool col_ok = rl < a.R[a.k_loop];
    for (int row = row0; row < row0 + 64 / HALVES; row += 4, of += 4 * sl) {
      if (col_ok && bl * 64 + row < a.R[a.k_lane]) ((gout_t)a.out)[of] = tile[row][col];
    }
  }
}

using WsumFn = void (*)(WsumArgs);

static WsumFn wsum_pick(const WsumArgs& a) {
  if (!a.use_box) return k_wsum<false, 0>;
  switch (a.cls ? a.em : 0) {
    case 3: return k_wsum<true, 3>;
    case 5: return k_wsum<true, 5>;
    case 8: return k_wsum<true, 8>;
    default: return k_wsum<true, 0>;
  }
}

hipError_t wsum_prepare() {
  for (WsumFn f : {k_wsum<true, 0>, k_wsum<true, 3>, k_wsum<true, 5>, k_wsum<true, 8>}) {
    hipError_t e = hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       2 * kWsumBoxMaxBytes + 256);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t wsum_launch(const WsumArgs& a, int64_t blocks, hipStream_t stream) {
  // the box, one spill slot per lane, then the row offsets
  const size_t lds = a.use_box ? (size_t)(a.box_elems + 64 + a.box_rows) * 4 : 0;
  hipLaunchKernelGGL(wsum_pick(a), dim3((unsigned)blocks), dim3(256), lds, stream, a);
  return hipGetLastError();
}

}  // namespace aol
