// Fused horizontal + vertical polyphase downscaler for gfx950.
//
// Sec. III of the paper: the downscaler is a horizontal filter over every
// line followed by a vertical filter over every column, repeated for every
// frame and colour plane; Sec. III-A: each filter is a repetitive task whose
// elementary tasks are independent. Sec. III-B (performance tuning): data
// exchanged between consecutive tasks should not make extra trips. Here both
// filters of one 2-D tile of repetitions run in one workgroup and the
// intermediate frame stays in LDS.
//
// Both passes are small dense products on the matrix cores. For a tile, an
// output block of 16 outputs along an axis reads a window of input elements;
// window x coefficients is D = A * B with
//   horizontal: A = 16 input lines x K input columns (pixels), B = K x 16 taps
//   vertical:   A = 16 intermediate columns x K intermediate lines (LDS), B = taps
// so every lane's A operand is 16 contiguous bytes of one line (a 128-bit
// load). The coefficient operands are prepared on the host in lane order.
// The 16x16 accumulator leaves each lane with 4 consecutive rows of one
// column, which is written to LDS transposed (Z^T[column][line]) so the
// vertical pass reads 16 contiguous bytes as well.
//
// Integer path: pixels enter the i8 MFMA as x ^ 0x80 = x - 128 and the
// missing 128*sum(c) is added back before the round-shift; taps beyond
// int8 range are carried as lo + 128*hi in two products. int32 accumulation
// makes the result exact. Float path: bf16/fp16 MFMA with fp32 accumulate;
// the intermediate is stored as a hi/lo pair of 16-bit values.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aol_internal.h"

namespace aol {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int pmod(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

// 16 contiguous bytes of row `row` starting at element `col`, wrapping
// modulo `w` elements (Array-OL tilers index modulo the array shape).
template <int ESIZE>
__device__ __forceinline__ v4i load_chunk(const uint8_t* row, int col, int w, int vec) {
  constexpr int E = 16 / ESIZE;
  if (vec && col >= 0 && col + E <= w) {
    return *reinterpret_cast<const v4i*>(row + (int64_t)col * ESIZE);
  }
  v4i r;
  if constexpr (ESIZE == 1) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) v |= (uint32_t)row[pmod(col + 4 * d + e, w)] << (8 * e);
      r[d] = (int)v;
    }
  } else {
    const uint16_t* r16 = reinterpret_cast<const uint16_t*>(row);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t lo = r16[pmod(col + 2 * d, w)];
      uint32_t hi = r16[pmod(col + 2 * d + 1, w)];
      r[d] = (int)(lo | (hi << 16));
    }
  }
  return r;
}

__device__ __forceinline__ v4i to_i8(v4i x) {
  const int m = (int)0x80808080u;
  return v4i{x[0] ^ m, x[1] ^ m, x[2] ^ m, x[3] ^ m};
}

template <int ELEM>
__device__ __forceinline__ v4f mfma16(v4i a, v4i b, v4f c) {
  if constexpr (ELEM == kBF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  }
}

// clamp(floor((acc + bias) / 256), 0, 255) for four accumulators, packed
// little-endian. The sum is clamped to [0, 65535] first, so its byte 1 is
// the result, and v_perm gathers those bytes. (Written this way on purpose:
// a clamp after the shift lets the compiler pick v_ashr_pk_u8_i32 for two of
// the lanes and then OR the full register, whose upper half still holds the
// sign bits of a negative sum.)
__device__ __forceinline__ uint32_t quant4(v4i acc, int bias) {
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = acc[i] + bias;
    x[i] = (uint32_t)min(max(v, 0), 65535);
  }
  const uint32_t lo = __builtin_amdgcn_perm(x[1], x[0], 0x0c0c0501u);  // bytes: x0.b1, x1.b1, 0, 0
  const uint32_t hi = __builtin_amdgcn_perm(x[3], x[2], 0x05010c0cu);  // bytes: 0, 0, x2.b1, x3.b1
  return lo | hi;
}

template <int ELEM>
__device__ __forceinline__ uint16_t to16(float x) {
  if constexpr (ELEM == kBF16) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);
  } else {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
  }
}

template <int ELEM>
__device__ __forceinline__ float from16(uint16_t x) {
  if constexpr (ELEM == kBF16) {
    return __uint_as_float((uint32_t)x << 16);
  } else {
    return (float)__builtin_bit_cast(_Float16, x);
  }
}

// One tile: tx-th group of TRx repetitions along lines, ty-th group of TRy
// along columns, of plane `pl` in frame `frame`.
template <int ELEM, int NW>
__device__ __forceinline__ void fused_tile(const FusedArgs& a, const PlaneArg& pl, int frame, int tx, int ty,
                                           uint8_t* lds) {
  constexpr int ES = (ELEM == kU8) ? 1 : 2;  // bytes per element
  constexpr int E = 16 / ES;                 // elements per 16-byte chunk
  const AxisBand* __restrict__ hb = a.hb;
  const AxisBand* __restrict__ vb = a.vb;
  const v4i* __restrict__ hfrag = reinterpret_cast<const v4i*>(a.hfrag);
  const v4i* __restrict__ vfrag = reinterpret_cast<const v4i*>(a.vfrag);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;  // K group of this lane
  const int n = lane & 15;  // M/N index of this lane

  const int R0x = tx * hb->tr, R0y = ty * vb->tr;
  const int nRx = min(hb->tr, pl.rx - R0x);
  const int nRy = min(vb->tr, pl.ry - R0y);
  const int Lz = vb->q * (nRy - 1) + vb->span;  // intermediate lines this tile needs
  const int zrow0 = vb->q * R0y + vb->s_min;    // frame line of intermediate line 0
  const int nbH = (hb->p * nRx + 15) >> 4;      // 16-column blocks of the intermediate
  const int nbV = (vb->p * nRy + 15) >> 4;      // 16-line blocks of the output
  const int a0 = hb->q * R0x + hb->s_min - hb->delta;  // frame column of chunk 0 (chunk aligned)
  const int zp = a.zpitch;
  const int split = (ELEM == kU8) ? hb->split : 0;
  const int vsplit = (ELEM == kU8) ? vb->split : 0;

  const uint8_t* src = reinterpret_cast<const uint8_t*>(pl.in) + ((int64_t)frame * pl.in_fstride) * ES;

  // ---------------- horizontal pass: z[line][col] for all intermediate lines of the tile
  for (int mb = wave; mb < a.z_mblocks; mb += NW) {
    const int j = mb * 16 + n;  // intermediate line of this lane's A row
    if (mb * 16 >= Lz) {
      if constexpr (ELEM != kU8) {  // keep unused lines finite: they meet zero taps in the vertical pass
        for (int b = 0; b < nbH; ++b) {
          uint16_t* zh = reinterpret_cast<uint16_t*>(lds) + (16 * b + n) * zp + mb * 16 + 4 * g;
          *reinterpret_cast<uint2*>(zh) = uint2{0u, 0u};
          *reinterpret_cast<uint2*>(zh + a.zrows * zp) = uint2{0u, 0u};
        }
      }
      continue;
    }
    const bool rowok = j < Lz;
    const int grow = pmod(zrow0 + j, pl.h);
    const uint8_t* rp = src + (int64_t)grow * pl.in_pitch * ES;
    for (int b = 0; b < nbH; ++b) {
      const int c0 = hb->chunk0[b];
      const int nk = hb->nk[b];
      const int fb = hb->frag[b];
      if constexpr (ELEM == kU8) {
        v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
        for (int kb = 0; kb < nk; ++kb) {
          const int col = a0 + (c0 + 4 * kb + g) * E;
          v4i av = rowok ? to_i8(load_chunk<1>(rp, col, pl.w, pl.vec_in)) : v4i{0, 0, 0, 0};
          if (split) {
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, hfrag[((fb + kb) * 2) * 64 + lane], acc, 0, 0, 0);
            acch = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, hfrag[((fb + kb) * 2 + 1) * 64 + lane], acch, 0, 0, 0);
          } else {
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, hfrag[(fb + kb) * 64 + lane], acc, 0, 0, 0);
          }
        }
        if (split) acc = acc + acch * 128;
        const uint32_t z4 = quant4(acc, hb->bias[b * 16 + n]);
        *reinterpret_cast<uint32_t*>(lds + (16 * b + n) * zp + mb * 16 + 4 * g) = z4;
      } else {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int kb = 0; kb < nk; ++kb) {
          const int col = a0 + (c0 + 4 * kb + g) * E;
          v4i av = rowok ? load_chunk<2>(rp, col, pl.w, pl.vec_in) : v4i{0, 0, 0, 0};
          acc = mfma16<ELEM>(av, hfrag[(fb + kb) * 64 + lane], acc);
        }
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hi[i] = to16<ELEM>(acc[i]);
          lo[i] = to16<ELEM>(acc[i] - from16<ELEM>(hi[i]));
        }
        uint16_t* zh = reinterpret_cast<uint16_t*>(lds) + (16 * b + n) * zp + mb * 16 + 4 * g;
        *reinterpret_cast<uint2*>(zh) = uint2{(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
        *reinterpret_cast<uint2*>(zh + a.zrows * zp) =
            uint2{(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
      }
    }
  }
  __syncthreads();

  // ---------------- vertical pass: y[line][col] from the intermediate in LDS
  const int orow0 = vb->p * R0y;
  const int ocol0 = hb->p * R0x;
  uint8_t* dst = reinterpret_cast<uint8_t*>(pl.out) + ((int64_t)frame * pl.out_fstride) * (ELEM == kU8 ? 1 : 4);
  for (int job = wave; job < nbH * nbV; job += NW) {
    const int cb = job % nbH;
    const int b = job / nbH;
    const int c0 = vb->chunk0[b];
    const int nk = vb->nk[b];
    const int fb = vb->frag[b];
    const int orow = orow0 + 16 * b + n;
    const int col = ocol0 + 16 * cb + 4 * g;
    if constexpr (ELEM == kU8) {
      v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
      const uint8_t* zr = lds + (16 * cb + n) * zp;
      for (int kb = 0; kb < nk; ++kb) {
        v4i av = to_i8(*reinterpret_cast<const v4i*>(zr + (c0 + 4 * kb + g) * 16));
        if (vsplit) {
          acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, vfrag[((fb + kb) * 2) * 64 + lane], acc, 0, 0, 0);
          acch = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, vfrag[((fb + kb) * 2 + 1) * 64 + lane], acch, 0, 0, 0);
        } else {
          acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, vfrag[(fb + kb) * 64 + lane], acc, 0, 0, 0);
        }
      }
      if (vsplit) acc = acc + acch * 128;
      if (orow < pl.mh) {
        const uint32_t y4 = quant4(acc, vb->bias[b * 16 + n]);
        uint8_t* op = dst + (int64_t)orow * pl.out_pitch + col;
        if (pl.vec_out && col + 4 <= pl.mw) {
          *reinterpret_cast<uint32_t*>(op) = y4;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (col + i < pl.mw) op[i] = (uint8_t)(y4 >> (8 * i));
        }
      }
    } else {
      v4f acc = {0.f, 0.f, 0.f, 0.f};
      const uint16_t* zr = reinterpret_cast<const uint16_t*>(lds) + (16 * cb + n) * zp;
      for (int kb = 0; kb < nk; ++kb) {
        const int off = (c0 + 4 * kb + g) * 8;
        const v4i bv = vfrag[(fb + kb) * 64 + lane];
        acc = mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + off), bv, acc);
        acc = mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + a.zrows * zp + off), bv, acc);
      }
      if (orow < pl.mh) {
        float* op = reinterpret_cast<float*>(dst) + (int64_t)orow * pl.out_pitch + col;
        if (pl.vec_out && col + 4 <= pl.mw) {
          *reinterpret_cast<v4f*>(op) = acc;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (col + i < pl.mw) op[i] = acc[i];
        }
      }
    }
  }
}

// Maps a workgroup to a tile. Workgroups are dealt to the 8 XCDs round-robin;
// the remap gives each XCD one contiguous run of tiles (column-major inside
// a plane), so tiles that share halo lines run on the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int xcd = bid & 7, k = bid >> 3;
  const int q8 = n >> 3, r8 = n & 7;
  return xcd * q8 + min(xcd, r8) + k;
}

template <int ELEM, int NW>
__global__ __launch_bounds__(NW * 64) void k_fused(FusedArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int t_all = xcd_remap(blockIdx.x, a.total_tiles);
  const int frame = t_all / a.tiles_per_frame;
  int t = t_all - frame * a.tiles_per_frame;
  int pi = 0;
#pragma unroll
  for (int k = 1; k < kMaxPlanes; ++k)
    if (k < a.n_planes && t >= a.pl[k].tile_base) pi = k;
  const PlaneArg& pl = a.pl[pi];
  t -= pl.tile_base;
  const int tx = t / pl.tiles_y;
  const int ty = t - tx * pl.tiles_y;
  fused_tile<ELEM, NW>(a, pl, frame, tx, ty, lds);
}

constexpr int kWaves = 4;

hipError_t fused_prepare(int elem, size_t lds_bytes) {
  const void* f = elem == kU8 ? (const void*)k_fused<kU8, kWaves>
                 : elem == kBF16 ? (const void*)k_fused<kBF16, kWaves>
                                 : (const void*)k_fused<kFP16, kWaves>;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t fused_launch(int elem, const FusedArgs& a, size_t lds_bytes, hipStream_t stream) {
  dim3 grid(a.total_tiles), block(kWaves * 64);
  if (elem == kU8)
    hipLaunchKernelGGL((k_fused<kU8, kWaves>), grid, block, lds_bytes, stream, a);
  else if (elem == kBF16)
    hipLaunchKernelGGL((k_fused<kBF16, kWaves>), grid, block, lds_bytes, stream, a);
  else
    hipLaunchKernelGGL((k_fused<kFP16, kWaves>), grid, block, lds_bytes, stream, a);
  return hipGetLastError();
}

}  // namespace aol
