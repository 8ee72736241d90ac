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
//   vertical:   A = 16 intermediate columns x K intermediate lines, B = taps
// so every lane's A operand is 16 contiguous bytes of one line. The
// coefficient operands are prepared on the host in lane order. The 16x16
// accumulator leaves each lane with 4 consecutive rows of one column, which
// is written to LDS transposed (Z^T[column][line]) so the vertical pass
// reads 16 contiguous bytes as well.
//
// Integer path: pixels enter the i8 MFMA as x ^ 0x80 = x - 128 and the
// missing 128*sum(c) is added back before the round-shift; taps beyond
// int8 range are carried as lo + 128*hi in two products. int32 accumulation
// makes the result exact. Float path: bf16/fp16 MFMA with fp32 accumulate;
// the intermediate is stored as a hi/lo pair of 16-bit values.
//
// Schedule: a persistent grid. Each workgroup stages the coefficient
// fragments in LDS once, then walks its tiles: while the matrix cores work on
// tile i (input tile in LDS), the 16-byte loads of tile i+1 are in flight in
// registers; they are committed to LDS between the two passes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aol_internal.h"

namespace aol {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Workgroup barrier that orders LDS only. __syncthreads() also waits for
// every outstanding global load (vmcnt(0)), which would drain the register
// prefetch of the next input lines at each barrier; here global loads stay in
// flight until their registers are consumed.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int pmod(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

// Element-wise gather of one 16-byte chunk with the column taken modulo the
// line length (borders, misaligned rows). Kept out of line: it is rare and
// would otherwise multiply the register footprint of the unrolled loads.
template <int ESIZE>
__device__ __attribute__((noinline)) v4i load_chunk_wrap(const uint8_t* row, int col, int w) {
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

// 16 contiguous bytes of row `row` starting at element `col`, wrapping
// modulo `w` elements (Array-OL tilers index modulo the array shape).
template <int ESIZE>
__device__ __forceinline__ v4i load_chunk(const uint8_t* row, int col, int w, int vec) {
  constexpr int E = 16 / ESIZE;
  if (vec && col >= 0 && col + E <= w) {
    return *reinterpret_cast<const v4i*>(row + (int64_t)col * ESIZE);
  }
  return load_chunk_wrap<ESIZE>(row, col, w);
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

__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
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

// Geometry of one tile (all values uniform across the workgroup).
struct TileGeo {
  int pi, frame;
  int R0x, R0y, nRx, nRy;
  int Lz;     // intermediate lines the tile needs (= input lines staged)
  int zrow0;  // frame line of intermediate line 0
  int a0;     // frame column of input chunk 0
  int nch;    // input chunks per line the tile needs
  int nbH, nbV;
};

__device__ __forceinline__ TileGeo tile_geo(const FusedArgs& a, const AxisBand* __restrict__ hb,
                                            const AxisBand* __restrict__ vb, int t) {
  TileGeo g;
  g.frame = t / a.tiles_per_frame;
  int tt = t - g.frame * a.tiles_per_frame;
  int pi = 0;
#pragma unroll
  for (int k = 1; k < kMaxPlanes; ++k)
    if (k < a.n_planes && tt >= a.pl[k].tile_base) pi = k;
  g.pi = pi;
  const PlaneArg& pl = a.pl[pi];
  tt -= pl.tile_base;
  int tx, ty;
  if (a.walk == 0) {  // row-major: consecutive tiles are horizontal neighbours
    ty = tt / pl.tiles_x;
    tx = tt - ty * pl.tiles_x;
  } else {  // column-major: consecutive tiles are vertical neighbours
    tx = tt / pl.tiles_y;
    ty = tt - tx * pl.tiles_y;
  }
  g.R0x = tx * hb->tr;
  g.R0y = ty * vb->tr;
  g.nRx = min(hb->tr, pl.rx - g.R0x);
  g.nRy = min(vb->tr, pl.ry - g.R0y);
  g.Lz = vb->q * (g.nRy - 1) + vb->span;
  g.zrow0 = vb->q * g.R0y + vb->s_min;
  g.a0 = hb->q * g.R0x + hb->s_min - hb->delta;
  const int E = hb->chunk_elems;
  g.nch = min(a.xchunks, (hb->delta + hb->q * (g.nRx - 1) + hb->span + E - 1) / E);
  g.nbH = (hb->p * g.nRx + 15) >> 4;
  g.nbV = (vb->p * g.nRy + 15) >> 4;
  return g;
}

template <int ELEM, int SLOTS>
struct Stager {
  static constexpr int ES = (ELEM == kU8) ? 1 : 2;
  static constexpr int E = 16 / ES;
  v4i pre[SLOTS];

  // Issue the 16-byte loads of a tile's input window (lines x chunks) into
  // registers; round r covers the lines of slots r*SLOTS .. r*SLOTS+SLOTS-1.
  __device__ __forceinline__ void issue(const FusedArgs& a, const TileGeo& g, int wave, int lr, int lc, int r) {
    const PlaneArg& pl = a.pl[g.pi];
    const uint8_t* src = reinterpret_cast<const uint8_t*>(pl.in) + ((int64_t)g.frame * pl.in_fstride) * ES;
    const int rpl = a.rows_per_load;
    const bool lane_ok = lr < rpl && lc < g.nch;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int row = ((r * SLOTS + s) * kWaves + wave) * rpl + lr;
      v4i v = {0, 0, 0, 0};
      if (lane_ok && row < g.Lz) {
        int grow = g.zrow0 + row;
        if (grow < 0 || grow >= pl.h) grow = pmod(grow, pl.h);
        const uint8_t* rp = src + (int64_t)grow * pl.in_pitch * ES;
        v = load_chunk<ES>(rp, g.a0 + lc * E, pl.w, pl.vec_in);
      }
      pre[s] = v;
    }
  }

  // Write the staged chunks into the LDS input tile (chunks past the tile's
  // need are written as zeros so every element the matrix cores read is finite).
  __device__ __forceinline__ void commit(const FusedArgs& a, const TileGeo& g, int wave, int lr, int lc,
                                         uint8_t* xs, int r) {
    const int rpl = a.rows_per_load;
    if (lr >= rpl) return;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int row = ((r * SLOTS + s) * kWaves + wave) * rpl + lr;
      if (row < g.Lz) *reinterpret_cast<v4i*>(xs + row * a.xpitch + lc * 16) = pre[s];
    }
  }
};

template <int ELEM, bool SPLIT, int MAXK>
__device__ __forceinline__ void h_pass(const FusedArgs& a, const TileGeo& g, const AxisBand* __restrict__ hb,
                                       const uint8_t* lds, int wave, int lane) {
  const int gq = lane >> 4, n = lane & 15;
  constexpr bool split = (ELEM == kU8) && SPLIT;
  const v4i* fr = reinterpret_cast<const v4i*>(lds + a.lds.frag_h);
  const int* bias = reinterpret_cast<const int*>(lds + a.lds.bias_h);
  const uint8_t* xs = lds + a.lds.x;
  uint8_t* zs = const_cast<uint8_t*>(lds) + a.lds.z;
  const int zp = a.zpitch;
  const int nmb = a.z_mblocks;
  const int nmb_need = (g.Lz + 15) >> 4;
  int cur_b = -1, c0 = 0, nk = 0, bz = 0;
  v4i B[MAXK], Bh[split ? MAXK : 1];
  // jobs (b, mb) in order b-major, mb-minor; wave w takes jobs w, w+4, ...
  int b = 0, mb = wave;
  while (mb >= nmb) {
    mb -= nmb;
    ++b;
  }
  for (; b < g.nbH; mb += kWaves) {
    while (mb >= nmb) {
      mb -= nmb;
      ++b;
    }
    if (b >= g.nbH) break;
    if (mb >= nmb_need) {
      if constexpr (ELEM != kU8) {  // unused lines stay finite: they meet zero taps in the vertical pass
        uint16_t* zh = reinterpret_cast<uint16_t*>(zs) + (16 * b + n) * zp + mb * 16 + 4 * gq;
        *reinterpret_cast<uint2*>(zh) = uint2{0u, 0u};
        *reinterpret_cast<uint2*>(zh + a.zrows * zp) = uint2{0u, 0u};
      }
      continue;
    }
    if (b != cur_b) {
      cur_b = b;
      c0 = hb->chunk0[b];
      nk = hb->nk[b];
      const int fb = hb->frag[b];
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          if constexpr (split) {
            B[kb] = fr[((fb + kb) * 2) * 64 + lane];
            Bh[kb] = fr[((fb + kb) * 2 + 1) * 64 + lane];
          } else {
            B[kb] = fr[(fb + kb) * 64 + lane];
          }
        }
      }
      if constexpr (ELEM == kU8) bz = bias[b * 16 + n];
    }
    const int row = mb * 16 + n;
    const bool rowok = row < g.Lz;
    const uint8_t* xr = xs + row * a.xpitch;
    if constexpr (ELEM == kU8) {
      v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          const v4i av = rowok ? to_i8(*reinterpret_cast<const v4i*>(xr + (c0 + 4 * kb + gq) * 16)) : v4i{0, 0, 0, 0};
          acc = mfma_i8(av, B[kb], acc);
          if constexpr (split) acch = mfma_i8(av, Bh[kb], acch);
        }
      }
      if constexpr (split) acc = acc + acch * 128;
      *reinterpret_cast<uint32_t*>(zs + (16 * b + n) * zp + mb * 16 + 4 * gq) = quant4(acc, bz);
    } else {
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          const v4i av = rowok ? *reinterpret_cast<const v4i*>(xr + (c0 + 4 * kb + gq) * 16) : v4i{0, 0, 0, 0};
          acc = mfma16<ELEM>(av, B[kb], acc);
        }
      }
      uint16_t hi[4], lo[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        hi[i] = to16<ELEM>(acc[i]);
        lo[i] = to16<ELEM>(acc[i] - from16<ELEM>(hi[i]));
      }
      uint16_t* zh = reinterpret_cast<uint16_t*>(zs) + (16 * b + n) * zp + mb * 16 + 4 * gq;
      *reinterpret_cast<uint2*>(zh) = uint2{(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
      *reinterpret_cast<uint2*>(zh + a.zrows * zp) =
          uint2{(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
    }
  }
}

template <int ELEM, bool SPLIT, int MAXK>
__device__ __forceinline__ void v_pass(const FusedArgs& a, const TileGeo& g, const AxisBand* __restrict__ hb,
                                       const AxisBand* __restrict__ vb, const uint8_t* lds, int wave, int lane) {
  const int gq = lane >> 4, n = lane & 15;
  constexpr bool split = (ELEM == kU8) && SPLIT;
  const v4i* fr = reinterpret_cast<const v4i*>(lds + a.lds.frag_v);
  const int* bias = reinterpret_cast<const int*>(lds + a.lds.bias_v);
  const uint8_t* zs = lds + a.lds.z;
  const int zp = a.zpitch;
  const PlaneArg& pl = a.pl[g.pi];
  const int orow0 = vb->p * g.R0y;
  const int ocol0 = hb->p * g.R0x;
  // outputs of this tile only: a 16-wide block can run past the tile's last
  // repetition into rows/columns that belong to the neighbouring tile
  const int row_end = min(pl.mh, orow0 + vb->p * g.nRy);
  const int col_end = min(pl.mw, ocol0 + hb->p * g.nRx);
  uint8_t* dst = reinterpret_cast<uint8_t*>(pl.out) + ((int64_t)g.frame * pl.out_fstride) * (ELEM == kU8 ? 1 : 4);
  int cur_b = -1, c0 = 0, nk = 0, bz = 0;
  v4i B[MAXK], Bh[split ? MAXK : 1];
  // jobs (b, cb) in order b-major, cb-minor; wave w takes jobs w, w+4, ...
  int b = 0, cb = wave;
  for (;; cb += kWaves) {
    while (cb >= g.nbH) {
      cb -= g.nbH;
      ++b;
    }
    if (b >= g.nbV) break;
    if (b != cur_b) {
      cur_b = b;
      c0 = vb->chunk0[b];
      nk = vb->nk[b];
      const int fb = vb->frag[b];
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          if constexpr (split) {
            B[kb] = fr[((fb + kb) * 2) * 64 + lane];
            Bh[kb] = fr[((fb + kb) * 2 + 1) * 64 + lane];
          } else {
            B[kb] = fr[(fb + kb) * 64 + lane];
          }
        }
      }
      if constexpr (ELEM == kU8) bz = bias[b * 16 + n];
    }
    const int orow = orow0 + 16 * b + n;
    const int col = ocol0 + 16 * cb + 4 * gq;
    if constexpr (ELEM == kU8) {
      v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
      const uint8_t* zr = zs + (16 * cb + n) * zp;
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          const v4i av = to_i8(*reinterpret_cast<const v4i*>(zr + (c0 + 4 * kb + gq) * 16));
          acc = mfma_i8(av, B[kb], acc);
          if constexpr (split) acch = mfma_i8(av, Bh[kb], acch);
        }
      }
      if constexpr (split) acc = acc + acch * 128;
      if (orow < row_end) {
        const uint32_t y4 = quant4(acc, bz);
        uint8_t* op = dst + (int64_t)orow * pl.out_pitch + col;
        if (pl.vec_out && col + 4 <= col_end) {
          *reinterpret_cast<uint32_t*>(op) = y4;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (col + i < col_end) op[i] = (uint8_t)(y4 >> (8 * i));
        }
      }
    } else {
      v4f acc = {0.f, 0.f, 0.f, 0.f};
      const uint16_t* zr = reinterpret_cast<const uint16_t*>(zs) + (16 * cb + n) * zp;
#pragma unroll
      for (int kb = 0; kb < MAXK; ++kb) {
        if (kb < nk) {
          const int off = (c0 + 4 * kb + gq) * 8;
          acc = mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + off), B[kb], acc);
          acc = mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + a.zrows * zp + off), B[kb], acc);
        }
      }
      if (orow < row_end) {
        float* op = reinterpret_cast<float*>(dst) + (int64_t)orow * pl.out_pitch + col;
        if (pl.vec_out && col + 4 <= col_end) {
          *reinterpret_cast<v4f*>(op) = acc;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (col + i < col_end) op[i] = acc[i];
        }
      }
    }
  }
}

// Tiles of workgroup `wg` of `G`: one contiguous run of the row-major tile
// order, so each tile's left halo lines were fetched by the same workgroup
// for its previous tile and are still in cache.
struct TileWalk {
  int next, end;
  __device__ __forceinline__ TileWalk(int wg, int G, int n) {
    const int q = n / G, r = n - q * G;
    next = wg * q + min(wg, r);
    end = next + q + (wg < r ? 1 : 0);
  }
  __device__ __forceinline__ int pop() {
    const int t = next < end ? next : -1;
    ++next;
    return t;
  }
};

template <int ELEM, bool SPLIT, int SLOTS, int MAXK>
__global__ __launch_bounds__(kWaves * 64) void k_fused(FusedArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const AxisBand* __restrict__ hb = a.hb;
  const AxisBand* __restrict__ vb = a.vb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps job loops scalar
  const int lr = lane / a.xchunks, lc = lane - lr * a.xchunks;

  TileWalk walk(blockIdx.x, gridDim.x, a.total_tiles);
  int t = walk.pop();
  if (t < 0) return;

  // coefficient fragments and biases of both axes, once per workgroup
  {
    const int nh = hb->nfrag * 64, nv = vb->nfrag * 64;
    const v4i* gh = reinterpret_cast<const v4i*>(a.hfrag);
    const v4i* gv = reinterpret_cast<const v4i*>(a.vfrag);
    v4i* sh = reinterpret_cast<v4i*>(lds + a.lds.frag_h);
    v4i* sv = reinterpret_cast<v4i*>(lds + a.lds.frag_v);
    for (int i = tid; i < nh; i += kWaves * 64) sh[i] = gh[i];
    for (int i = tid; i < nv; i += kWaves * 64) sv[i] = gv[i];
    if constexpr (ELEM == kU8) {
      int* bh = reinterpret_cast<int*>(lds + a.lds.bias_h);
      int* bv = reinterpret_cast<int*>(lds + a.lds.bias_v);
      for (int i = tid; i < hb->nblk * 16; i += kWaves * 64) bh[i] = hb->bias[i];
      for (int i = tid; i < vb->nblk * 16; i += kWaves * 64) bv[i] = vb->bias[i];
    }
  }

  Stager<ELEM, SLOTS> st;
  TileGeo g = tile_geo(a, hb, vb, t);
  for (int r = 0; r < a.load_rounds; ++r) {
    st.issue(a, g, wave, lr, lc, r);
    st.commit(a, g, wave, lr, lc, lds + a.lds.x, r);
  }
  lds_barrier();

  while (true) {
    const int tn = walk.pop();
    TileGeo gn;
    if (tn >= 0) {
      gn = tile_geo(a, hb, vb, tn);
      st.issue(a, gn, wave, lr, lc, 0);  // in flight during this tile's passes
    }
    h_pass<ELEM, SPLIT, MAXK>(a, g, hb, lds, wave, lane);
    lds_barrier();  // input tile consumed, intermediate complete
    if (tn >= 0) {
      st.commit(a, gn, wave, lr, lc, lds + a.lds.x, 0);
      for (int r = 1; r < a.load_rounds; ++r) {  // tiles larger than one round of loads
        st.issue(a, gn, wave, lr, lc, r);
        st.commit(a, gn, wave, lr, lc, lds + a.lds.x, r);
      }
    }
    v_pass<ELEM, SPLIT, MAXK>(a, g, hb, vb, lds, wave, lane);
    lds_barrier();  // intermediate consumed, next input tile staged
    if (tn < 0) break;
    g = gn;
  }
}

// Kernel instances: element type x split taps x prefetch depth x K-steps.
// The plan picks the smallest instance its band and tile fit.
using KernelFn = void (*)(FusedArgs);
constexpr int kSlotOpts[2] = {6, kMaxSlots};
constexpr int kKOpts[2] = {2, kMaxK};

template <int ELEM, bool SPLIT>
static KernelFn pick2(int si, int ki) {
  if (si == 0) return ki == 0 ? k_fused<ELEM, SPLIT, kSlotOpts[0], kKOpts[0]> : k_fused<ELEM, SPLIT, kSlotOpts[0], kKOpts[1]>;
  return ki == 0 ? k_fused<ELEM, SPLIT, kSlotOpts[1], kKOpts[0]> : k_fused<ELEM, SPLIT, kSlotOpts[1], kKOpts[1]>;
}

static KernelFn pick(int elem, bool split, int slots, int maxk) {
  const int si = slots <= kSlotOpts[0] ? 0 : 1;
  const int ki = maxk <= kKOpts[0] ? 0 : 1;
  if (elem == kU8) return split ? pick2<kU8, true>(si, ki) : pick2<kU8, false>(si, ki);
  if (elem == kBF16) return pick2<kBF16, false>(si, ki);
  return pick2<kFP16, false>(si, ki);
}

hipError_t fused_prepare(int elem, bool split, int slots, int maxk, size_t lds_bytes, int* wg_per_cu) {
  const void* f = (const void*)pick(elem, split, slots, maxk);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  int n = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kWaves * 64, lds_bytes);
  if (e != hipSuccess) return e;
  *wg_per_cu = n;
  return hipSuccess;
}

hipError_t fused_launch(int elem, bool split, int slots, int maxk, const FusedArgs& a, int grid, size_t lds_bytes,
                        hipStream_t stream) {
  hipLaunchKernelGGL(pick(elem, split, slots, maxk), dim3(grid), dim3(kWaves * 64), lds_bytes, stream, a);
  return hipGetLastError();
}

}  // namespace aol
