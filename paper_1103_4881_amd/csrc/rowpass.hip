// One polyphase pass along rows with a transposed output, for gfx950.
//
// The two filters of the downscaler (Sec. III: horizontal filter over every
// line, then vertical filter over every column) as two separate kernels
// exchanging the intermediate frame through HBM, like the paper's separate
// per-component tasks connected by frame arrays (Sec. III-A). Both passes are
// the same operation: filter every row of a uint8 array along the row
// (polyphase, ratio p/q, modulo wrap) and write the result transposed.
//
//   horizontal pass: X[h][w]    -> Z^T[mw][h]  (Z^T row = one column of Z)
//   vertical pass:   Z^T[mw][h] -> Y[mh][mw]   (transposing again gives Y)
//
// A tile is 128 rows (8 waves x 16) by 16 output blocks of 16. Each wave
// loads, for each block, one 16-byte chunk per lane straight from memory
// (16 rows x the block's window) and runs the block on the matrix cores
// (v_mfma_i32_16x16x64_i8 on x ^ 0x80, 128*sum(c) + 128 restored in the
// accumulator, taps beyond int8 split lo + 128*hi). Each lane's four rows
// of one output go, as one 32-bit word, into the tile's transposed outputs
// in LDS; the workgroup then writes each output row's 128 bytes as whole
// 16-byte stores (the direct per-lane words were 16-byte fragments of many
// rows, and the passes ran at a fifth of the memory's bandwidth).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aol_internal.h"
#include "rowpass.h"

namespace aol {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

#define RP_CONST __attribute__((address_space(4)))

__device__ __forceinline__ int rp_mod(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

// 16 bytes of a circular row starting at element x (any x), byte by byte.
__device__ __attribute__((noinline)) v4i rp_gather(const uint8_t* row, int x, int n) {
  v4i r;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    uint32_t v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) v |= (uint32_t)row[rp_mod(x + 4 * d + e, n)] << (8 * e);
    r[d] = (int)v;
  }
  return r;
}

// clamp(floor(acc / 256), 0, 255) x 4 (the rounding 128 is in acc), packed.
// Clamped before the shift so no packed shift can mix in sign bits.
__device__ __forceinline__ uint32_t rp_quant4(v4i acc) {
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = (uint32_t)min(max(acc[i], 0), 65535);
  return __builtin_amdgcn_perm(x[1], x[0], 0x0c0c0501u) | __builtin_amdgcn_perm(x[3], x[2], 0x05010c0cu);
}

__device__ __forceinline__ v4i rp_to_i8(v4i x) {
  const int m = (int)0x80808080u;
  return v4i{x[0] ^ m, x[1] ^ m, x[2] ^ m, x[3] ^ m};
}

}  // namespace

// SPLIT: coefficient operands as lo + 128*hi pairs; KM: largest K-step count
// of a block (4 chunks of 16 elements each).
template <bool SPLIT, int KM>
__global__ __launch_bounds__(kRowPassThreads) void k_rowpass(RowPassArgs A) {
  // blocks in flight per iteration (eight for one K-step measured slower: the
  // registers cost more waves than the extra loads win)
  constexpr int NJ = (SPLIT || KM > 2) ? 2 : 4;
  // the tile's outputs, transposed: row k = output 16*b0 + k, one byte per input row
  __shared__ __attribute__((aligned(16))) uint8_t tile_t[kRowPassBlocks * 16][kRowPassTilePitch];
  // Workgroups go to the 8 XCDs in turn (workgroup g on XCD g mod 8), each
  // XCD with its own L2: the workgroups of one XCD take consecutive tiles,
  // so the neighbouring tiles of a row of tiles, which read the same lines at
  // their edges, run one after the other on one XCD and fetch those lines
  // once. The grid is a multiple of 8; tiles past the last are empty.
  const int G8 = gridDim.x / 8, wg = blockIdx.x;
  const int tile = (wg % 8) * G8 + wg / 8;
  if (tile >= A.total_tiles) return;
  const int frame = tile / A.tiles_per_frame;
  int t = tile - frame * A.tiles_per_frame;
  int pi = 0;
  while (pi + 1 < A.n_planes && t >= A.pl[pi + 1].tile_base) ++pi;
  const RowPassPlane P = A.pl[pi];
  t -= P.tile_base;
  const int rt = t / P.blk_tiles, bt = t - rt * P.blk_tiles;  // neighbouring tiles along a row of tiles
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
  const int tile_row0 = rt * kRowPassRows;
  const int row0 = tile_row0 + wave * 16;
  const int b0 = bt * kRowPassBlocks, b1 = min(b0 + kRowPassBlocks, P.nblocks);
  if (row0 < P.rows) {  // whole wave
    const int row = min(row0 + n, P.rows - 1);  // rows past the end load the last one; never stored
    const uint8_t* src = P.in + (int64_t)frame * P.in_fstride + (int64_t)row * P.in_pitch;
    const RP_CONST AxisBand* band = (const RP_CONST AxisBand*)A.band;
    const int p = band->p;
    const int pq16 = 16 * band->q;  // input elements per period of 16 repetitions
    const uint8_t* frag = (const uint8_t*)A.frag + lane * 16;
    for (int b = b0; b < b1; b += NJ) {
      v4i a[NJ][KM], c[NJ][KM], ch[NJ][SPLIT ? KM : 1];
      int nk[NJ], lb[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int bj = min(b + j, b1 - 1);  // a missing block repeats the last one; not kept
        const int per = bj / p;
        lb[j] = bj - per * p;
        nk[j] = __builtin_amdgcn_readfirstlane(band->nk[lb[j]]);
        const int xs = per * pq16 + A.x0 + 16 * band->chunk0[lb[j]];  // element of the window's first chunk
        const int fb = band->frag[lb[j]];
        const bool inside = P.vec_in && xs >= 0 && xs + 64 * nk[j] <= P.n;  // uniform
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (k > 0 && k >= nk[j]) break;  // uniform
          const int x = xs + 16 * (4 * k + g);
          a[j][k] = rp_to_i8(inside ? *reinterpret_cast<const v4i*>(src + x) : rp_gather(src, x, P.n));
          if constexpr (SPLIT) {
            c[j][k] = *reinterpret_cast<const v4i*>(frag + (2 * (fb + k)) * 1024);
            ch[j][k] = *reinterpret_cast<const v4i*>(frag + (2 * (fb + k) + 1) * 1024);
          } else {
            c[j][k] = *reinterpret_cast<const v4i*>(frag + (fb + k) * 1024);
          }
        }
      }
      v4i acc[NJ], acch[SPLIT ? NJ : 1];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int bias = band->bias[lb[j] * 16 + n];  // 128 * sum(c) + 128 of output n of the block
        acc[j] = v4i{bias, bias, bias, bias};
        if constexpr (SPLIT) acch[j] = v4i{0, 0, 0, 0};
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          if (k > 0 && k >= nk[j]) continue;  // uniform: the block's own K-steps only
          acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], c[j][k], acc[j], 0, 0, 0);
          if constexpr (SPLIT) acch[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], ch[j][k], acch[j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if (j > 0 && b + j >= b1) break;
        v4i r = acc[j];
        if constexpr (SPLIT) r = r + acch[j] * 128;
        // rows row0+4g .. +3 of output 16*(b+j) + n
        *reinterpret_cast<uint32_t*>(&tile_t[16 * (b + j - b0) + n][16 * wave + 4 * g]) = rp_quant4(r);
      }
    }
  }
  __syncthreads();
  // The tile's transposed outputs: each output row gets the tile's rows as
  // one contiguous run (a whole 128-byte line when the tile is full).
  const int nrows = min(kRowPassRows, P.rows - tile_row0);
  const int nout = min(16 * b1, P.m) - 16 * b0;
  uint8_t* dst = P.out + (int64_t)frame * P.out_fstride + (int64_t)(16 * b0) * P.out_pitch + tile_row0;
  for (int idx = threadIdx.x; idx < nout * (kRowPassRows / 16); idx += kRowPassThreads) {
    const int k = idx / (kRowPassRows / 16), c = idx - k * (kRowPassRows / 16);
    const int r0 = 16 * c;
    if (r0 >= nrows) continue;
    uint8_t* op = dst + (int64_t)k * P.out_pitch + r0;
    const v4i v = *reinterpret_cast<const v4i*>(&tile_t[k][r0]);
    if (r0 + 16 <= nrows && P.vec_out == 16) {
      *reinterpret_cast<v4i*>(op) = v;
    } else if (r0 + 16 <= nrows && P.vec_out == 4) {
#pragma unroll
      for (int i = 0; i < 4; ++i) reinterpret_cast<uint32_t*>(op)[i] = (uint32_t)v[i];
    } else {
      for (int e = 0; e < 16 && r0 + e < nrows; ++e) op[e] = (uint8_t)((uint32_t)v[e >> 2] >> (8 * (e & 3)));
    }
  }
}

typedef void (*RowPassFn)(RowPassArgs);

static RowPassFn rowpass_pick(bool split, int kmax) {
  if (split) return kmax <= 1 ? k_rowpass<true, 1> : kmax <= 2 ? k_rowpass<true, 2> : k_rowpass<true, 4>;
  return kmax <= 1 ? k_rowpass<false, 1> : kmax <= 2 ? k_rowpass<false, 2> : k_rowpass<false, 4>;
}

hipError_t rowpass_launch(bool split, int kmax, const RowPassArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(rowpass_pick(split, kmax), dim3(grid), dim3(kRowPassThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace aol
