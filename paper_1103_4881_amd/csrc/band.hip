// Band-scheduled fused downscaler for gfx950 (integer and float forms).
//
// Both filters of the downscaler (Sec. III: horizontal filter over every
// line, then vertical filter over every column, per frame and colour plane;
// Sec. III-A: one independent elementary task per repetition) in one kernel,
// scheduled so that every input byte is fetched once:
//
//  * one workgroup owns a column band of a plane (its full width whenever it
//    fits, else bands of whole 16-repetition periods whose edges read one
//    halo chunk) and walks a segment of repetitions down it, 16 input lines
//    per step, with coalesced 16-byte loads of whole band lines; the modulo
//    wrap at the plane's left and right edges reads the same line;
//  * the horizontal pass turns the 16 staged lines into 16 intermediate lines
//    for every 16-column block on the matrix cores and writes them,
//    transposed, into a ring in LDS spanning the band;
//  * whenever the ring holds the window of the next 16 output lines, the
//    vertical pass runs on it and stores them; the vertical halo never leaves
//    the chip. Loads run two steps ahead in registers.
//
// Operands: A = 16 lines x (4 chunks of 16 bytes per K-step), one chunk per
// lane; B = the coefficients of one 16-output block in lane order, prepared
// on the host for one period of 16 repetitions (q chunks, p blocks) and
// reused for every period. Integer: i8 MFMA on x ^ 0x80, 128*sum(c) restored
// before the round-shift, taps beyond int8 split lo + 128*hi, int32
// accumulation (exact), uint8 intermediate. Float: bf16/fp16 MFMA with fp32
// accumulation, the intermediate kept as a hi/lo pair of 16-bit values, fp32
// output.
//
// Work comes from a unit list (stream, column band, segment) of one frame,
// repeated over frames: the same kernel serves one plan's planes x frames and
// a batch of video streams with different sizes and filters, whose units are
// ordered so that a workgroup's consecutive units mostly share a filter.
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

constexpr int kBandWaves = kBandThreads / 64;

__device__ __forceinline__ int bpmod(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

template <int ES>
__device__ __attribute__((noinline)) v4i b_load_chunk_wrap(const uint8_t* row, int col, int w) {
  v4i r;
  if constexpr (ES == 1) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) v |= (uint32_t)row[bpmod(col + 4 * d + e, w)] << (8 * e);
      r[d] = (int)v;
    }
  } else {
    const uint16_t* r16 = reinterpret_cast<const uint16_t*>(row);
#pragma unroll
    for (int d = 0; d < 4; ++d)
      r[d] = (int)((uint32_t)r16[bpmod(col + 2 * d, w)] | ((uint32_t)r16[bpmod(col + 2 * d + 1, w)] << 16));
  }
  return r;
}

__device__ __forceinline__ v4i b_to_i8(v4i x) {
  const int m = (int)0x80808080u;
  return v4i{x[0] ^ m, x[1] ^ m, x[2] ^ m, x[3] ^ m};
}

// clamp(floor((acc + bias) / 256), 0, 255) x 4, packed. Clamped before the
// shift on purpose: a clamp after it lets the compiler use v_ashr_pk_u8_i32
// and OR the register's stale upper half into the neighbouring bytes.
__device__ __forceinline__ uint32_t b_quant4(v4i acc, int bias) {
  uint32_t x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = (uint32_t)min(max(acc[i] + bias, 0), 65535);
  return __builtin_amdgcn_perm(x[1], x[0], 0x0c0c0501u) | __builtin_amdgcn_perm(x[3], x[2], 0x05010c0cu);
}

template <int ELEM>
__device__ __forceinline__ v4f b_mfma16(v4i a, v4i b, v4f c) {
  if constexpr (ELEM == kBF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  }
}

template <int ELEM>
__device__ __forceinline__ uint32_t b_pack2(float x, float y) {
  if constexpr (ELEM == kBF16) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x) | ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)y) << 16);
  } else {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)y) << 16);
  }
}

template <int ELEM>
__device__ __forceinline__ float b_lo16(uint32_t v) {
  if constexpr (ELEM == kBF16) return __uint_as_float(v << 16);
  else return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu));
}

template <int ELEM>
__device__ __forceinline__ float b_hi16(uint32_t v) {
  if constexpr (ELEM == kBF16) return __uint_as_float(v & 0xFFFF0000u);
  else return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}

// Per-unit geometry (uniform across the workgroup).
struct BandUnitGeo {
  const uint8_t* src;
  uint8_t* dst;
  int zrow0, Lz, M, NBV, a0, orow0, ocol0, row_end, col_end, nbh;
  int vec_in, vec_out;
};

template <int ELEM, int SLOTS>
struct BandStager {
  static constexpr int ES = ELEM == kU8 ? 1 : 2;
  static constexpr int E = 16 / ES;
  v4i pre[SLOTS];
  // the 16 lines of step m, chunks of the band, into registers; slot s of
  // thread t is chunk t + s*threads of the step, line-major
  __device__ __forceinline__ void issue(const BandStream& S, const BandUnitGeo& u, int m, int tid) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int idx = tid + s * kBandThreads;
      const int r = (int)__umulhi((uint32_t)idx, S.nch_magic);  // idx / nch
      const int c = idx - r * S.nch;
      v4i v = {0, 0, 0, 0};
      if (r < 16 && 16 * m + r < u.Lz) {
        int grow = u.zrow0 + 16 * m + r;
        if (grow < 0 || grow >= S.h) grow = bpmod(grow, S.h);
        const uint8_t* rp = u.src + (int64_t)grow * S.in_pitch * ES;
        int col = u.a0 + c * E;
        if (u.vec_in) {
          // whole chunks of a circular line: a wrapped chunk is another chunk
          while (col < 0) col += S.w;
          while (col >= S.w) col -= S.w;
          v = *reinterpret_cast<const v4i*>(rp + (int64_t)col * ES);
        } else {
          v = b_load_chunk_wrap<ES>(rp, col, S.w);
        }
      }
      pre[s] = v;
    }
  }
  __device__ __forceinline__ void commit(const BandStream& S, uint8_t* xs, int tid) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int idx = tid + s * kBandThreads;
      const int r = (int)__umulhi((uint32_t)idx, S.nch_magic);
      const int c = idx - r * S.nch;
      if (r < 16) *reinterpret_cast<v4i*>(xs + r * S.xpitch + c * 16) = pre[s];
    }
  }
};

template <int ELEM, int SLOTS, bool SPLIT>
__global__ __launch_bounds__(kBandThreads) void k_band(BandLaunch L) {
  constexpr int ES = ELEM == kU8 ? 1 : 2;
  constexpr int E = 16 / ES;
  constexpr bool split = (ELEM == kU8) && SPLIT;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, n = lane & 15;

  BandStager<ELEM, SLOTS> s0, s1;
  const AxisBand* cur_hb = nullptr;
  for (int u = blockIdx.x; u < L.total_units; u += gridDim.x) {
    const int frame = u / L.units_per_frame;
    const BandUnit U = L.units[u - frame * L.units_per_frame];
    // by value: kept in scalar registers instead of being re-read from memory
    // after every global store (the compiler cannot rule out aliasing)
    const BandStream S = L.streams[U.stream];
    const AxisBand* __restrict__ hb = S.hb;
    const AxisBand* __restrict__ vb = S.vb;
    uint8_t* xs = lds + S.lds_x;
    uint8_t* zs = lds + S.lds_z;
    const v4i* fh = reinterpret_cast<const v4i*>(lds + S.lds_fh);
    const v4i* fv = reinterpret_cast<const v4i*>(lds + S.lds_fv);
    const int* bh = reinterpret_cast<const int*>(lds + S.lds_bh);
    const int* bv = reinterpret_cast<const int*>(lds + S.lds_bv);
    const int RM = S.ring - 1;

    lds_barrier();  // the previous unit is done with LDS
    if (hb != cur_hb) {  // coefficient operands and biases of this stream's filter
      cur_hb = hb;
      const v4i* gh = reinterpret_cast<const v4i*>(S.hfrag);
      const v4i* gv = reinterpret_cast<const v4i*>(S.vfrag);
      for (int i = tid; i < hb->nfrag * 64; i += kBandThreads) const_cast<v4i*>(fh)[i] = gh[i];
      for (int i = tid; i < vb->nfrag * 64; i += kBandThreads) const_cast<v4i*>(fv)[i] = gv[i];
      if constexpr (ELEM == kU8) {
        for (int i = tid; i < hb->nblk * 16; i += kBandThreads) const_cast<int*>(bh)[i] = hb->bias[i];
        for (int i = tid; i < vb->nblk * 16; i += kBandThreads) const_cast<int*>(bv)[i] = vb->bias[i];
      }
    }

    BandUnitGeo G;
    {
      const void* pin = L.ptr_table ? L.ptr_table[2 * S.ptr] : L.ptrs[2 * S.ptr];
      void* pout = L.ptr_table ? L.ptr_table[2 * S.ptr + 1] : const_cast<void*>(L.ptrs[2 * S.ptr + 1]);
      const int64_t fin = L.ptr_table ? 0 : L.fstride[2 * S.ptr];
      const int64_t fout = L.ptr_table ? 0 : L.fstride[2 * S.ptr + 1];
      G.src = reinterpret_cast<const uint8_t*>(pin) + (int64_t)frame * fin * ES;
      G.dst = reinterpret_cast<uint8_t*>(pout) + (int64_t)frame * fout * (ELEM == kU8 ? 1 : 4);
      const int R0x = U.xb * S.xreps, R0y = U.sy * S.seg;
      const int nRx = min(S.xreps, S.rx - R0x);
      const int nRy = min(S.seg, S.ry - R0y);
      G.Lz = vb->q * (nRy - 1) + vb->span;
      G.zrow0 = vb->q * R0y + vb->s_min;
      G.M = (G.Lz + 15) >> 4;
      G.NBV = (vb->p * nRy + 15) >> 4;
      G.a0 = hb->q * R0x + hb->s_min - hb->delta;
      G.orow0 = vb->p * R0y;
      G.ocol0 = hb->p * R0x;
      G.row_end = min(S.mh, G.orow0 + vb->p * nRy);
      G.col_end = min(S.mw, G.ocol0 + hb->p * nRx);
      G.nbh = (hb->p * nRx + 15) >> 4;
      G.vec_in = S.vec_in && L.aligned;
      G.vec_out = S.vec_out && L.aligned;
    }

    // loads run AHEAD steps ahead: two stagers alternate (narrow lines), or
    // one stager is issued at the start of a step and committed in its middle
    constexpr int AHEAD = SLOTS <= 2 ? 2 : 1;
    int B = 0;  // next vertical block
    auto step = [&](int m, BandStager<ELEM, SLOTS>& mine, BandStager<ELEM, SLOTS>& other) {
      if (m + AHEAD < G.M) mine.issue(S, G, m + AHEAD, tid);
      // ---- horizontal pass: 16 intermediate lines of every 16-column block
      if constexpr (ELEM == kU8 && !split && SLOTS <= 2) {
        // two blocks per iteration: their LDS reads and MFMAs overlap
        for (int b0 = wave; b0 < G.nbh; b0 += 2 * kBandWaves) {
          const int b1 = b0 + kBandWaves;
          const bool two = b1 < G.nbh;
          const int per0 = b0 / hb->nblk, lb0 = b0 - per0 * hb->nblk;
          const int per1 = two ? b1 / hb->nblk : per0, lb1 = two ? b1 - per1 * hb->nblk : lb0;
          const int c00 = hb->chunk0[lb0] + per0 * hb->q, c01 = hb->chunk0[lb1] + per1 * hb->q;
          const int nk0 = hb->nk[lb0], nk1 = two ? hb->nk[lb1] : 0;
          const int fb0 = hb->frag[lb0], fb1 = hb->frag[lb1];
          const uint8_t* xr = xs + n * S.xpitch;
          v4i acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
          const int nkm = nk0 > nk1 ? nk0 : nk1;
          for (int kb = 0; kb < nkm; ++kb) {
            v4i a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
            if (kb < nk0) a0 = *reinterpret_cast<const v4i*>(xr + (c00 + 4 * kb + g) * 16);
            if (kb < nk1) a1 = *reinterpret_cast<const v4i*>(xr + (c01 + 4 * kb + g) * 16);
            if (kb < nk0) acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(b_to_i8(a0), fh[(fb0 + kb) * 64 + lane], acc0, 0, 0, 0);
            if (kb < nk1) acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(b_to_i8(a1), fh[(fb1 + kb) * 64 + lane], acc1, 0, 0, 0);
          }
          const int zoff = (16 * m + 4 * g) & RM;
          *reinterpret_cast<uint32_t*>(zs + (16 * b0 + n) * S.rpitch + zoff) = b_quant4(acc0, bh[lb0 * 16 + n]);
          if (two) *reinterpret_cast<uint32_t*>(zs + (16 * b1 + n) * S.rpitch + zoff) = b_quant4(acc1, bh[lb1 * 16 + n]);
        }
      } else
      for (int b = wave; b < G.nbh; b += kBandWaves) {
        const int per = b / hb->nblk, lb = b - per * hb->nblk;
        const int c0 = hb->chunk0[lb] + per * (hb->q * 16 / E);  // a period is 16q elements
        const int nk = hb->nk[lb], fb = hb->frag[lb];
        const uint8_t* xr = xs + n * S.xpitch;
        if constexpr (ELEM == kU8) {
          v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
          for (int kb = 0; kb < nk; ++kb) {
            const v4i av = b_to_i8(*reinterpret_cast<const v4i*>(xr + (c0 + 4 * kb + g) * 16));
            if constexpr (split) {
              acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fh[((fb + kb) * 2) * 64 + lane], acc, 0, 0, 0);
              acch = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fh[((fb + kb) * 2 + 1) * 64 + lane], acch, 0, 0, 0);
            } else {
              acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fh[(fb + kb) * 64 + lane], acc, 0, 0, 0);
            }
          }
          if constexpr (split) acc = acc + acch * 128;
          *reinterpret_cast<uint32_t*>(zs + (16 * b + n) * S.rpitch + ((16 * m + 4 * g) & RM)) =
              b_quant4(acc, bh[lb * 16 + n]);
        } else {
          v4f acc = {0.f, 0.f, 0.f, 0.f};
          for (int kb = 0; kb < nk; ++kb)
            acc = b_mfma16<ELEM>(*reinterpret_cast<const v4i*>(xr + (c0 + 4 * kb + g) * 16), fh[(fb + kb) * 64 + lane], acc);
          // hi/lo pair: hi = round(z), lo = round(z - hi)
          const uint32_t h01 = b_pack2<ELEM>(acc[0], acc[1]);
          const uint32_t h23 = b_pack2<ELEM>(acc[2], acc[3]);
          const uint32_t l01 = b_pack2<ELEM>(acc[0] - b_lo16<ELEM>(h01), acc[1] - b_hi16<ELEM>(h01));
          const uint32_t l23 = b_pack2<ELEM>(acc[2] - b_lo16<ELEM>(h23), acc[3] - b_hi16<ELEM>(h23));
          uint8_t* zp = zs + (16 * b + n) * S.rpitch + ((16 * m + 4 * g) & RM) * 2;
          *reinterpret_cast<uint2*>(zp) = uint2{h01, h23};
          *reinterpret_cast<uint2*>(zp + S.zhalf) = uint2{l01, l23};
        }
      }
      lds_barrier();  // staging consumed, intermediate lines written
      if (m + 1 < G.M) other.commit(S, xs, tid);
      // ---- vertical blocks whose window is complete
      const int have = min(G.Lz, 16 * (m + 1));
      while (B < G.NBV) {
        const int per = B / vb->nblk, lb = B - per * vb->nblk;
        const int need = min(G.Lz, vb->wend[lb] + 16 * per * vb->q);
        if (need > have) break;
        const int c0 = vb->chunk0[lb] + per * (vb->q * 16 / E);  // chunks of E intermediate lines
        const int nk = vb->nk[lb], fb = vb->frag[lb];
        const int orow = G.orow0 + 16 * B + n;
        for (int cb = wave; cb < G.nbh; cb += kBandWaves) {
          const uint8_t* zr = zs + (16 * cb + n) * S.rpitch;
          const int col = G.ocol0 + 16 * cb + 4 * g;
          if constexpr (ELEM == kU8) {
            v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
            for (int kb = 0; kb < nk; ++kb) {
              const v4i av = b_to_i8(*reinterpret_cast<const v4i*>(zr + (((c0 + 4 * kb + g) * 16) & RM)));
              if constexpr (split) {
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fv[((fb + kb) * 2) * 64 + lane], acc, 0, 0, 0);
                acch = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fv[((fb + kb) * 2 + 1) * 64 + lane], acch, 0, 0, 0);
              } else {
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fv[(fb + kb) * 64 + lane], acc, 0, 0, 0);
              }
            }
            if constexpr (split) acc = acc + acch * 128;
            if (orow < G.row_end) {
              const uint32_t y4 = b_quant4(acc, bv[lb * 16 + n]);
              uint8_t* op = G.dst + (int64_t)orow * S.out_pitch + col;
              if (G.vec_out && col + 4 <= G.col_end) {
                *reinterpret_cast<uint32_t*>(op) = y4;
              } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  if (col + i < G.col_end) op[i] = (uint8_t)(y4 >> (8 * i));
              }
            }
          } else {
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            for (int kb = 0; kb < nk; ++kb) {
              const int off = (((c0 + 4 * kb + g) * 8) & RM) * 2;
              const v4i bf = fv[(fb + kb) * 64 + lane];
              acc = b_mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + off), bf, acc);
              acc = b_mfma16<ELEM>(*reinterpret_cast<const v4i*>(zr + S.zhalf + off), bf, acc);
            }
            if (orow < G.row_end) {
              float* op = reinterpret_cast<float*>(G.dst) + (int64_t)orow * S.out_pitch + col;
              if (G.vec_out && col + 4 <= G.col_end) {
                *reinterpret_cast<v4f*>(op) = acc;
              } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  if (col + i < G.col_end) op[i] = acc[i];
              }
            }
          }
        }
        ++B;
      }
      lds_barrier();  // ring reads of this step done, next staging committed
    };

    if constexpr (ELEM != kU8) {
      // float ring starts at zero so the zero taps of a block's padding never meet a NaN
      for (int i = tid; i < (S.nbh * 16 * S.rpitch) / 16; i += kBandThreads) {
        reinterpret_cast<v4i*>(zs)[i] = v4i{0, 0, 0, 0};
        reinterpret_cast<v4i*>(zs + S.zhalf)[i] = v4i{0, 0, 0, 0};
      }
    }
    s0.issue(S, G, 0, tid);
    if (AHEAD == 2 && G.M > 1) s1.issue(S, G, 1, tid);
    s0.commit(S, xs, tid);
    lds_barrier();
    if constexpr (AHEAD == 2) {
      for (int m = 0; m < G.M; m += 2) {
        step(m, s0, s1);
        if (m + 1 < G.M) step(m + 1, s1, s0);
      }
    } else {
      for (int m = 0; m < G.M; ++m) step(m, s0, s0);
    }
  }
}

using BandFn = void (*)(BandLaunch);

template <int ELEM>
static BandFn band_pick_e(int slots, bool split) {
  if (slots <= 2) return split ? k_band<ELEM, 2, true> : k_band<ELEM, 2, false>;
  return split ? k_band<ELEM, 4, true> : k_band<ELEM, 4, false>;
}

static BandFn band_pick(int elem, int slots, bool split) {
  if (elem == kU8) return band_pick_e<kU8>(slots, split);
  if (elem == kBF16) return band_pick_e<kBF16>(slots, false);
  return band_pick_e<kFP16>(slots, false);
}

hipError_t band_prepare(int elem, int slots, bool split, size_t lds_bytes, int* wg_per_cu) {
  const void* f = (const void*)band_pick(elem, slots, split);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, f, kBandThreads, lds_bytes);
}

hipError_t band_launch(int elem, int slots, bool split, const BandLaunch& L, int grid, size_t lds_bytes,
                       hipStream_t stream) {
  hipLaunchKernelGGL(band_pick(elem, slots, split), dim3(grid), dim3(kBandThreads), lds_bytes, stream, L);
  return hipGetLastError();
}

// Writes up to 128 device pointers, passed by value, into a device table:
// the pointer update of a batch is an ordinary stream-ordered launch, so it
// can precede a captured graph launch without any host synchronisation.
struct PtrPack {
  void* p[128];
};

__global__ void k_set_ptrs(void** table, PtrPack pk, int n) {
  const int i = threadIdx.x;
  if (i < n) table[i] = pk.p[i];
}

hipError_t set_pointers_launch(void** table, const void* const* ptrs, int n, hipStream_t stream) {
  for (int base = 0; base < n; base += 128) {
    PtrPack pk;
    const int m = n - base < 128 ? n - base : 128;
    for (int i = 0; i < m; ++i) pk.p[i] = const_cast<void*>(ptrs[base + i]);
    hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(128), 0, stream, table + base, pk, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace aol
