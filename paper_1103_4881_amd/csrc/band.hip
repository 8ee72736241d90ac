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
//    the chip.
//
// The workgroup's waves have two roles. Waves 0-7 only load: they keep the
// next few steps of input lines in flight in registers and write step m+1
// into the staging lines while waves 8-15 run the vertical pass of step m.
// Waves 8-15 only compute and store. A gfx9 wave with both loads and stores
// outstanding can only wait for all of them, so mixing the roles would drain
// the prefetch at every step.
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
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
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
constexpr int kBandLoadWaves = kBandLoadThreads / 64;
static_assert(kBandMinHShares == 2 * (kBandWaves - kBandLoadWaves),
              "the compute waves alone can take every share of the horizontal pass");

// Shares of the horizontal pass each loading wave takes. None for the
// integer form with int8 taps and one K-step: there the loading waves' staging
// writes and loads queue behind each other at the LDS and the address unit
// right after every barrier, and matrix work behind that queue sets the
// step's length (measured 1.5-3 % faster without it). Otherwise two where the
// registers allow (the compute waves also run the vertical pass), else one
// (measured faster for the float forms and the split taps).
template <int ELEM, bool SPLIT, int KM, int SLOTS>
struct BandLoadShares {
  static constexpr int value = (ELEM == kU8 && !SPLIT && KM == 1) ? 0 : SPLIT || (KM >= 2 && SLOTS >= 4) ? 1 : 2;
};

// Pointers read from memory (descriptor and pointer tables) are generic to
// the compiler, and generic accesses become flat instructions, which count
// against both the vector-memory and the LDS counters: every wait for LDS
// would also wait for the prefetched input lines. Device data is therefore
// accessed through global (1) and constant (4) address-space pointers; the
// constant ones also let uniform descriptor reads go through the scalar unit.
#define AOL_GLOBAL __attribute__((address_space(1)))
#define AOL_CONST __attribute__((address_space(4)))
typedef const AOL_GLOBAL uint8_t* gsrc_t;
typedef AOL_GLOBAL uint8_t* gdst_t;
typedef const AOL_CONST AxisBand* cband_t;

// A copy of a device-resident descriptor read through the constant address
// space (scalar loads when the address is uniform).
template <class T>
__device__ __forceinline__ T load_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
  T v;
  const AOL_CONST uint32_t* src = (const AOL_CONST uint32_t*)p;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
  return v;
}

__device__ __forceinline__ int bpmod(int x, int m) {
  int r = x % m;
  return r < 0 ? r + m : r;
}

template <int ES>
__device__ __attribute__((noinline)) v4i b_load_chunk_wrap(gsrc_t row, int col, int w) {
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
    const AOL_GLOBAL uint16_t* r16 = (const AOL_GLOBAL uint16_t*)row;
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
  gsrc_t src;
  gdst_t dst;
  int zrow0, Lz, M, NBV, a0, orow0, ocol0, row_end, col_end, nbh;
  int vec_in, vec_out;
};

// Prefetch depth (staged steps in flight) for a number of chunks per loading
// lane and step: about 64 registers of input in flight per loading lane.
template <int SLOTS>
struct BandDepth {
  static constexpr int value = SLOTS <= 1 ? 8 : SLOTS <= 2 ? 6 : SLOTS <= 4 ? 3 : 1;
};

// The loading waves: each lane owns SLOTS chunks of every staged step (16
// input lines of the band, line-major), fixed for the unit. Every load is
// unconditional: a lane without a chunk, or a line past the unit's window,
// loads a line that another lane of the same step also loads (a cache hit,
// no extra HBM traffic), so the in-flight counts stay exact.
template <int ELEM, int SLOTS>
struct BandFeed {
  static constexpr int ES = ELEM == kU8 ? 1 : 2;
  static constexpr int E = 16 / ES;
  uint64_t p0[SLOTS];  // address of the chunk in step 0's line before the wrap (maybe outside the plane)
  int row[SLOTS];      // plane line of the chunk in step 0, before the wrap
  int xo[SLOTS];       // LDS byte offset of the chunk in the staging lines

  // lane's chunks: line rr and chunk c of the band line. A lane past the
  // last chunk loads and stores chunk 0 of line 15 again: the same bytes to
  // the same place, and no branch around the store, which would leave its
  // register's load outstanding on the other path.
  static __device__ __forceinline__ void chunk_of(const BandStream& S, int idx, int& rr, int& c) {
    rr = (int)__umulhi((uint32_t)idx, S.nch_magic);  // idx / nch
    c = idx - rr * S.nch;
    if (rr >= 16) { rr = 15; c = 0; }
  }

  // staging offsets of the lane's chunks (depend on the stream only)
  static __device__ __forceinline__ void offsets(const BandStream& S, int ltid, int (&xo)[SLOTS]) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      int rr, c;
      chunk_of(S, ltid + s * kBandLoadThreads, rr, c);
      xo[s] = rr * S.xpitch + c * 16;
    }
  }

  __device__ __forceinline__ void addresses(const BandStream& S, const BandUnitGeo& G, int ltid) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      int rr, c;
      chunk_of(S, ltid + s * kBandLoadThreads, rr, c);
      row[s] = G.zrow0 + rr;
      int cl = G.a0 + c * E;
      if (cl < 0 || cl >= S.w) cl = bpmod(cl, S.w);
      p0[s] = (uint64_t)(G.src + (int64_t)cl * ES) + (uint64_t)((int64_t)row[s] * S.in_pitch * ES);
    }
  }

  __device__ __forceinline__ void setup(const BandStream& S, const BandUnitGeo& G, int ltid) {
    addresses(S, G, ltid);
    offsets(S, ltid, xo);
  }

  __device__ __forceinline__ gsrc_t line(const BandStream& S, const BandUnitGeo& G, int m, int s) const {
    const int grow = bpmod(min(row[s] + 16 * m, G.zrow0 + G.Lz - 1), S.h);
    return G.src + (int64_t)grow * S.in_pitch * ES;
  }

  // Whole chunks of a circular line (a wrapped chunk is another chunk) of
  // step m of a unit with h plane lines, `pitch` bytes apart, and window
  // [zrow0, zrow0 + Lz). Straight-line code with the same loads on every
  // path, so the compiler's count of loads in flight stays exact: rows are
  // clamped and wrapped with arithmetic, and a step past the unit loads its
  // last line again. Interior steps (uniform test: all 16 lines inside the
  // plane and the window) advance each chunk's address by 16 lines; the
  // others clamp and wrap every line. Both paths load the same registers in
  // the same order.
  __device__ __forceinline__ void issue(v4i (&pre)[SLOTS], int h, int64_t pitch, int zrow0, int Lz, int m) const {
    const int top = zrow0 + 16 * m;
    if (top >= 0 && top + 16 <= h && 16 * m + 16 <= Lz) {
      const uint64_t adv = (uint64_t)(16 * m) * (uint64_t)pitch;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) pre[s] = *(const AOL_GLOBAL v4i*)(p0[s] + adv);
    } else {
      const int last = zrow0 + Lz - 1;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        // no per-lane branch between the loads: a divergent branch here
        // would make the compiler's load counts inexact
        const int gr = bpmod(min(row[s] + 16 * m, last), h);
        pre[s] = *(const AOL_GLOBAL v4i*)(p0[s] + (uint64_t)((int64_t)(gr - row[s]) * pitch));
      }
    }
  }

  // lines whose chunks are not whole chunks of the line: gathered element by
  // element with the wrap (a call, which waits for every load it issues)
  // and staged at once
  __device__ __forceinline__ void stage_gathered(const BandStream& S, const BandUnitGeo& G, int m, uint8_t* xs) const {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int col = (int)(((int64_t)(p0[s] - (uint64_t)G.src) - (int64_t)row[s] * S.in_pitch * ES) / ES);
      const v4i a = b_load_chunk_wrap<ES>(line(S, G, m, s), col, S.w);
      *reinterpret_cast<v4i*>(xs + xo[s]) = ELEM == kU8 ? b_to_i8(a) : a;
    }
  }

  // integer form: staged as signed bytes x - 128 (the matrix-core operand)
  static __device__ __forceinline__ void commit(const v4i (&pre)[SLOTS], const int (&xo)[SLOTS], uint8_t* xs) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s)
      *reinterpret_cast<v4i*>(xs + xo[s]) = ELEM == kU8 ? b_to_i8(pre[s]) : pre[s];
  }
};

// Horizontal pass of one step by one share. The pass is cut into shares:
// LS (none, one or two) for each loading wave and one or two for each
// compute wave (the compute waves also run the vertical pass). Each share takes
// blocks of one position lb within the period (shares v = lb, lb + nblk,
// ...: share v handles blocks lb + nblk*(v/nblk + gw*i), gw the shares of
// position lb), so its coefficient operands and biases are the same for all
// its blocks and stay in registers for the whole unit, and its blocks'
// staged chunks and ring rows advance by fixed strides. Writes 16
// intermediate lines of each of its 16-column blocks, transposed, into the
// ring.
// NB: blocks per iteration (operands in flight); CACHED: coefficient
// operands kept in registers where KM allows.
template <int ELEM, bool SPLIT, int KM, int NB, bool CACHED = true>
struct BandH {
  static constexpr int ES = ELEM == kU8 ? 1 : 2;
  static constexpr int E = 16 / ES;
  // operands of four K-steps would not fit in registers beside the vertical
  // pass's: read from LDS for every block instead
  static constexpr bool CACHE = CACHED && KM <= 2;
  v4i bf[CACHE ? KM : 1], bfh[SPLIT && CACHE ? KM : 1];  // coefficient operands of the wave's position
  const uint8_t* fl;  // lane's slot of the position's first fragment
  const uint8_t* bl;  // lane's bias
  v4i bq;                           // integer form: the rounding bias, every output of the lane's column
  int nbi, nk, astep, zstep, xbuf, zhalf;
  const uint8_t* xa;  // lane's A chunk of the wave's first block (staging buffer 0)
  uint8_t* zl;        // lane's ring row of the wave's first block

  // v: this share's index among the nv shares of the pass (none if v >= nv)
  __device__ __forceinline__ void setup(const BandStream& S, const BandUnitGeo& G, const uint8_t* lds, int v, int nv,
                                        int lane) {
    const cband_t hb = (cband_t)S.hb;
    const int g = lane >> 4, n = lane & 15;
    const int nblk = hb->nblk;
    const int lb = v % nblk, r = v / nblk;
    const int gw = (nv - lb + nblk - 1) / nblk;  // shares with this position
    const int b0 = lb + nblk * r, bstep = nblk * gw;
    // Wave-uniform by construction, and said so: values the compiler keeps
    // in vector registers make the block loop divergent, and a K-step skipped
    // under an EXEC mask is not skipped at all (MFMA ignores EXEC), so the
    // stale operands of an unused K-step would be added in.
    nbi = __builtin_amdgcn_readfirstlane(v < nv && b0 < G.nbh ? (G.nbh - b0 + bstep - 1) / bstep : 0);
    nk = __builtin_amdgcn_readfirstlane(hb->nk[lb]);
    const int fb = hb->frag[lb];
    fl = lds + S.lds_fh + lane * 16 + fb * (SPLIT ? 2048 : 1024);
    bl = lds + S.lds_bh + (lb * 16 + n) * 4;
    const int per0 = b0 / nblk;          // period of the first block
    const int pchunks = hb->q * 16 / E;  // chunks per period (16q elements)
    xa = lds + S.lds_x + n * S.xpitch + (hb->chunk0[lb] + per0 * pchunks + g) * 16;
    astep = __builtin_amdgcn_readfirstlane(gw * pchunks * 16);
    zl = const_cast<uint8_t*>(lds) + S.lds_z + (16 * b0 + n) * S.rpitch;
    zstep = __builtin_amdgcn_readfirstlane(16 * bstep * S.rpitch);
    xbuf = S.xbuf;
    zhalf = S.zhalf;
  }

  // the position's operands, once the unit's coefficients are in LDS (after
  // the unit's first barrier)
  __device__ __forceinline__ void load_operands() {
    if constexpr (CACHE) {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < nk || k == 0) {  // uniform; unused K-steps are never multiplied
          if constexpr (SPLIT) {
            bf[k] = *reinterpret_cast<const v4i*>(fl + (2 * k) * 1024);
            bfh[k] = *reinterpret_cast<const v4i*>(fl + (2 * k + 1) * 1024);
          } else {
            bf[k] = *reinterpret_cast<const v4i*>(fl + k * 1024);
          }
        }
      }
    }
    if constexpr (ELEM == kU8) {
      const int bias = *reinterpret_cast<const int*>(bl);
      bq = v4i{bias, bias, bias, bias};
    }
  }

  // zm: ring line of the step's first intermediate line; par: staging
  // buffer of the step
  __device__ __forceinline__ void run(int zm, int par, int g) const {
    const uint8_t* xm = xa + par * xbuf;
    uint8_t* zrow = zl + (zm + 4 * g) * ES;  // lane's 4 intermediate lines in its ring row
    for (int i = 0; i < nbi; i += NB) {
      v4i a[NB][KM];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int ii = min(i + j, nbi - 1);  // a missing block repeats the last one
#pragma unroll
        for (int k = 0; k < KM; ++k)
          if (k == 0 || k < nk) a[j][k] = *reinterpret_cast<const v4i*>(xm + ii * astep + 64 * k);
      }
      // all the products first (a missing block repeats the last one and
      // is not written), with no branch between them
      v4i acc[NB], acch[SPLIT ? NB : 1];
      v4f accf[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        acc[j] = bq;
        if constexpr (SPLIT) acch[j] = v4i{0, 0, 0, 0};
        accf[j] = v4f{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k > 0 && k >= nk) break;  // uniform: the position's own K-steps only
        v4i blo, bhi;
        if constexpr (CACHE) {
          blo = bf[k];
          if constexpr (SPLIT) bhi = bfh[k];
        } else if constexpr (SPLIT) {
          blo = *reinterpret_cast<const v4i*>(fl + (2 * k) * 1024);
          bhi = *reinterpret_cast<const v4i*>(fl + (2 * k + 1) * 1024);
        } else {
          blo = *reinterpret_cast<const v4i*>(fl + k * 1024);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if constexpr (ELEM == kU8) {
            acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], blo, acc[j], 0, 0, 0);
            if constexpr (SPLIT) acch[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], bhi, acch[j], 0, 0, 0);
          } else {
            accf[j] = b_mfma16<ELEM>(a[j][k], blo, accf[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j > 0 && i + j >= nbi) break;
        uint8_t* zp = zrow + (i + j) * zstep;
        if constexpr (ELEM == kU8) {
          v4i r = acc[j];
          if constexpr (SPLIT) r = r + acch[j] * 128;
          // kept as signed bytes z - 128, the vertical pass's operand
          *reinterpret_cast<uint32_t*>(zp) = b_quant4(r, 0) ^ 0x80808080u;
        } else {
          const v4f r = accf[j];
          // hi/lo pair: hi = round(z), lo = round(z - hi)
          const uint32_t h01 = b_pack2<ELEM>(r[0], r[1]);
          const uint32_t h23 = b_pack2<ELEM>(r[2], r[3]);
          const uint32_t l01 = b_pack2<ELEM>(r[0] - b_lo16<ELEM>(h01), r[1] - b_hi16<ELEM>(h01));
          const uint32_t l23 = b_pack2<ELEM>(r[2] - b_lo16<ELEM>(h23), r[3] - b_hi16<ELEM>(h23));
          *reinterpret_cast<uint2*>(zp) = uint2{h01, h23};
          *reinterpret_cast<uint2*>(zp + zhalf) = uint2{l01, l23};
        }
      }
    }
  }
};

// Stream descriptor and geometry of unit u (of the whole launch: units of
// one frame, repeated over frames).
template <int ELEM>
__device__ __forceinline__ void band_unit(const BandLaunch& L, int u, BandStream& S, BandUnitGeo& G) {
  constexpr int ES = ELEM == kU8 ? 1 : 2;
  const int frame = u / L.units_per_frame;
  const BandUnit U = load_const(L.units + (u - frame * L.units_per_frame));
  // by value: kept in scalar registers instead of being re-read from memory
  // after every global store (the compiler cannot rule out aliasing)
  S = load_const(L.streams + U.stream);
  const AOL_CONST uint64_t* table = (const AOL_CONST uint64_t*)L.ptr_table;
  const uint64_t pin = table ? table[2 * U.ptr] : (uint64_t)L.ptrs[2 * U.ptr];
  const uint64_t pout = table ? table[2 * U.ptr + 1] : (uint64_t)L.ptrs[2 * U.ptr + 1];
  const int64_t fin = L.ptr_table ? 0 : L.fstride[2 * U.ptr];
  const int64_t fout = L.ptr_table ? 0 : L.fstride[2 * U.ptr + 1];
  G.src = (gsrc_t)pin + (int64_t)frame * fin * ES;
  G.dst = (gdst_t)pout + (int64_t)frame * fout * (ELEM == kU8 ? 1 : 4);
  G.Lz = U.Lz;
  G.zrow0 = U.zrow0;
  G.M = U.M;
  G.NBV = U.NBV;
  G.a0 = U.a0;
  G.orow0 = U.orow0;
  G.ocol0 = U.ocol0;
  G.row_end = U.row_end;
  G.col_end = U.col_end;
  G.nbh = U.nbh;
  G.vec_in = S.vec_in && L.aligned;
  G.vec_out = L.aligned ? S.vec_out : 0;
}

// The workgroup's slot in the rounds. Workgroups are dispatched to the 8
// XCDs in turn (workgroup g on XCD g mod 8), each XCD with its own L2; when
// the launch groups items (column bands of one segment next to each other,
// frame-major), the workgroups of one XCD take consecutive slots, so the
// bands of a segment run on one XCD at the same time and the lines at their
// shared edges are fetched from memory once.
__device__ __forceinline__ int band_slot(const BandLaunch& L) {
  const int G = L.ngroups, g = (int)blockIdx.x - L.wg0;
  return (L.grouped && G % 8 == 0) ? (g % 8) * (G / 8) + g / 8 : g;
}

// Workgroup's share of the launch: positions [i0, i1) of its sequence of
// units. With a unit order (batches) the sequence is its slice of that
// table. Without one (downscale plans) the launch's items, the units of one
// frame most expensive first, each repeated over the frames (item x is unit
// x / n_frames of frame x mod n_frames), are dealt in rounds of one per
// workgroup, every other round in reverse order, so that each workgroup
// gets a similar mix of long and short units whatever the frame count.
__device__ __forceinline__ void band_share(const BandLaunch& L, int& i0, int& i1) {
  if (L.order) {
    const AOL_CONST int32_t* f = (const AOL_CONST int32_t*)L.first + ((int)blockIdx.x - L.wg0);
    i0 = f[0];
    i1 = f[1];
  } else {
    const int G = L.ngroups, g = band_slot(L);
    const int full = L.total_units / G, rem = L.total_units - full * G;
    const int pos = (full & 1) ? G - 1 - g : g;  // position in the last, partial round
    i0 = 0;
    i1 = full + (pos < rem ? 1 : 0);
  }
}

__device__ __forceinline__ int band_unit_at(const BandLaunch& L, int i) {
  if (L.order) return ((const AOL_CONST int32_t*)L.order)[i];
  const int G = L.ngroups, g = band_slot(L);
  const int x = i * G + ((i & 1) ? G - 1 - g : g);  // item of round i
  if (L.grouped) return x;  // frame-major items: frame * units_per_frame + unit
  const int unit = x / L.n_frames, frame = x - unit * L.n_frames;
  return frame * L.units_per_frame + unit;
}

// Stream descriptor of unit u (the loading waves need the next unit's
// staging offsets before its geometry).
__device__ __forceinline__ BandStream band_stream_of(const BandLaunch& L, int u) {
  const int frame = u / L.units_per_frame;
  const BandUnit U = load_const(L.units + (u - frame * L.units_per_frame));
  return load_const(L.streams + U.stream);
}

// The loading waves' read position: the unit and step whose lines the next
// issue loads, and the lane's chunk addresses in that unit. It runs D steps
// ahead of the staging and moves on to the workgroup's next unit at the end
// of one, so a unit's first lines are in flight while the previous one ends.
// Past the workgroup's last unit it stays on that unit's last line.
template <int ELEM, int SLOTS>
struct BandCursor {
  static constexpr int ES = ELEM == kU8 ? 1 : 2;
  BandFeed<ELEM, SLOTS> F;
  int i, i1, m, M, h, zrow0, Lz;  // position in the unit order, end of the workgroup's share
  int64_t pitch;  // bytes between plane lines

  __device__ __forceinline__ void at(const BandStream& S, const BandUnitGeo& G, int pos, int ltid) {
    F.addresses(S, G, ltid);
    i = pos;
    m = 0;
    M = G.M;
    h = S.h;
    zrow0 = G.zrow0;
    Lz = G.Lz;
    pitch = S.in_pitch * ES;
  }
  __device__ __forceinline__ void issue(v4i (&pre)[SLOTS]) const { F.issue(pre, h, pitch, zrow0, Lz, m); }
  __device__ __forceinline__ void advance(const BandLaunch& L, int ltid) {
    ++m;
    if (m == M && i + 1 < i1) {  // uniform; no loads on this path
      BandStream S;
      BandUnitGeo G;
      band_unit<ELEM>(L, band_unit_at(L, i + 1), S, G);
      at(S, G, i + 1, ltid);
    }
  }
};

// Loading waves (whole chunks): one pipeline over all the workgroup's units.
// Each step commits the next step's lines (maybe the next unit's first) into
// the staging buffer the compute waves are not reading, issues the loads D
// steps ahead, takes its LS shares of the horizontal pass (none where the
// compute waves take them all), and meets the compute waves at the step's
// barrier; a unit adds a barrier at its end (its LDS free) and one at the
// next unit's start (its coefficients in place).
// The staging buffer of a step is the parity of its index in the
// workgroup's sequence of steps. These waves issue no stores to memory and
// every iteration commits and re-issues one register set, so the loads in
// flight at the loop head are the same sets in the same order on entry and
// on the back edge, and their waits count exactly (on gfx9 a wave with loads
// and stores outstanding can only wait for all of them).
template <int ELEM, int SLOTS, int LS, class HP>
__device__ __forceinline__ void band_load_pipeline(const BandLaunch& L, uint8_t* lds, int tid, int wave, int lane) {
  constexpr int NV = LS * kBandLoadWaves + (kBandWaves - kBandLoadWaves);  // shares of the horizontal pass
  constexpr int D = BandDepth<SLOTS>::value;
  const int g = lane >> 4;
  int i, i1;  // position in the unit order, end of the workgroup's share
  band_share(L, i, i1);
  BandStream S;
  BandUnitGeo G;
  band_unit<ELEM>(L, band_unit_at(L, i), S, G);
  BandCursor<ELEM, SLOTS> C;
  C.i1 = i1;
  C.at(S, G, i, tid);
  int xo[SLOTS];
  BandFeed<ELEM, SLOTS>::offsets(S, tid, xo);
  HP H, H2;  // this wave's shares of the horizontal pass (H2: when LS is 2)
  if constexpr (LS > 0) H.setup(S, G, lds, wave, NV, lane);
  if constexpr (LS == 2) H2.setup(S, G, lds, wave + kBandLoadWaves, NV, lane);
  v4i pre[D][SLOTS];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    C.issue(pre[k]);
    C.advance(L, tid);
  }
  BandFeed<ELEM, SLOTS>::commit(pre[0], xo, lds + S.lds_x);  // step 0: buffer 0
  C.issue(pre[0]);
  C.advance(L, tid);
  lds_barrier();  // step 0 staged, the unit's coefficients in place
  if constexpr (LS > 0) H.load_operands();
  if constexpr (LS == 2) H2.load_operands();
  int m = 0, t = 0, zm = 0;  // step within the unit, step within the workgroup, ring line
  bool live = true;          // uniform: units left
  // Whole groups of D steps (the register set of a step is a constant once
  // unrolled). The loop is left only at the end of a group: an exit from
  // inside would reach the loop head, as the compiler lays it out, with
  // another set newest and make every wait there drain the prefetch. After
  // the last unit the group finishes without barriers or compute.
  for (;;) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int j = (k + 1) % D;
      const bool last = m + 1 == G.M;  // uniform
      if (last && i + 1 < i1)  // the next step is the next unit's first
        BandFeed<ELEM, SLOTS>::offsets(band_stream_of(L, band_unit_at(L, i + 1)), tid, xo);
      BandFeed<ELEM, SLOTS>::commit(pre[j], xo, lds + S.lds_x + ((t + 1) & 1) * S.xbuf);
      C.issue(pre[j]);
      C.advance(L, tid);
      if (live) {
        if constexpr (LS > 0) H.run(zm, t & 1, g);  // this wave's shares of step m's horizontal pass
        if constexpr (LS == 2) H2.run(zm, t & 1, g);
        zm = zm + 16 == S.ring ? 0 : zm + 16;
        lds_barrier();  // step m done with its buffer, the next step staged
        if (last) {
          lds_barrier();  // the compute waves are done with the unit's LDS
          ++i;
          live = i < i1;
          if (live) {
            band_unit<ELEM>(L, band_unit_at(L, i), S, G);
            if constexpr (LS > 0) H.setup(S, G, lds, wave, NV, lane);
            if constexpr (LS == 2) H2.setup(S, G, lds, wave + kBandLoadWaves, NV, lane);
            m = -1;
            zm = 0;
            lds_barrier();  // the unit's coefficients in place (its step 0 was staged before)
            if constexpr (LS > 0) H.load_operands();
            if constexpr (LS == 2) H2.load_operands();
          }
        }
      }
      ++m;
      ++t;
    }
    if (!live) break;
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): nothing left in flight
}

// Loading waves for lines that are gathered element by element: no
// prefetch, unit by unit (a call, which waits for every load it issues).
template <int ELEM, int SLOTS, int LS, class HP>
__device__ __forceinline__ void band_load_gathered(const BandLaunch& L, uint8_t* lds, int tid, int wave, int lane) {
  constexpr int NV = LS * kBandLoadWaves + (kBandWaves - kBandLoadWaves);
  const int g = lane >> 4;
  int t0 = 0;  // the unit's first step within the workgroup (staging buffer parity)
  int i0, i1;
  band_share(L, i0, i1);
  for (int i = i0; i < i1; ++i) {
    BandStream S;
    BandUnitGeo G;
    band_unit<ELEM>(L, band_unit_at(L, i), S, G);
    BandFeed<ELEM, SLOTS> F;
    F.setup(S, G, tid);
    HP H, H2;
    if constexpr (LS > 0) H.setup(S, G, lds, wave, NV, lane);
    if constexpr (LS == 2) H2.setup(S, G, lds, wave + kBandLoadWaves, NV, lane);
    uint8_t* xs = lds + S.lds_x;
    F.stage_gathered(S, G, 0, xs + (t0 & 1) * S.xbuf);
    lds_barrier();  // step 0 staged, the unit's coefficients in place
    if constexpr (LS > 0) H.load_operands();
    if constexpr (LS == 2) H2.load_operands();
    int zm = 0;
    for (int m = 0; m < G.M; ++m) {
      if (m + 1 < G.M) F.stage_gathered(S, G, m + 1, xs + ((t0 + m + 1) & 1) * S.xbuf);
      if constexpr (LS > 0) H.run(zm, (t0 + m) & 1, g);
      if constexpr (LS == 2) H2.run(zm, (t0 + m) & 1, g);
      zm = zm + 16 == S.ring ? 0 : zm + 16;
      lds_barrier();  // step m done with its buffer, step m+1 staged
    }
    lds_barrier();  // the compute waves are done with the unit's LDS
    t0 += G.M;
  }
}

// GATHER: an instance for launches with a line that is not made of whole
// 16-byte chunks (its width or pitch, or a pointer), whose loading waves
// gather elements; the other instances only stream whole chunks.
template <int ELEM, int SLOTS, bool SPLIT, int KM, bool GATHER>
__device__ __forceinline__ void band_body(const BandLaunch& L, uint8_t* lds) {
  constexpr int ES = ELEM == kU8 ? 1 : 2;
  constexpr int E = 16 / ES;
  constexpr bool split = (ELEM == kU8) && SPLIT;
  constexpr int NW = (kBandThreads - kBandLoadThreads) / 64;  // compute waves
  constexpr int NB = KM <= 2 && !split ? 4 : 1;               // vertical blocks per iteration (operands in flight)
  constexpr int LS = BandLoadShares<ELEM, split, KM, SLOTS>::value;  // horizontal shares per loading wave
  // horizontal blocks per iteration: all four where the compute waves take
  // the whole pass, else about two per share and step at the usual ratios
  constexpr int NBH = LS == 0 ? NB : (NB > 2 ? 2 : NB);
  constexpr int NBL = 1;  // the loading waves: one (their prefetch holds the registers; measured no slower)
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool loader = wave < kBandLoadThreads / 64;
  const int cw = wave - kBandLoadThreads / 64;  // compute wave index
  const int ctid = tid - kBandLoadThreads;
  const int g = lane >> 4, n = lane & 15;

  // The two roles loop over the same units separately, so that the loading
  // waves' code never has a store in flight.
  int i0, i1;
  band_share(L, i0, i1);
  if (loader) {
    if (i0 >= i1) return;
    // few blocks at a time in the horizontal pass: the prefetch holds the registers
    if constexpr (GATHER) band_load_gathered<ELEM, SLOTS, LS, BandH<ELEM, split, KM, 1>>(L, lds, tid, wave, lane);
    else band_load_pipeline<ELEM, SLOTS, LS, BandH<ELEM, split, KM, NBL>>(L, lds, tid, wave, lane);
    return;
  }

  cband_t cur_hb = nullptr;
  int t0 = 0;  // the unit's first step within the workgroup (staging buffer parity)
  for (int i = i0; i < i1; ++i) {
    BandStream S;
    BandUnitGeo G;
    band_unit<ELEM>(L, band_unit_at(L, i), S, G);
    const cband_t hb = (cband_t)S.hb;
    const cband_t vb = (cband_t)S.vb;
    uint8_t* zs = lds + S.lds_z;
    const uint8_t* fh = lds + S.lds_fh;
    const uint8_t* fv = lds + S.lds_fv;
    const uint8_t* bh = lds + S.lds_bh;
    const uint8_t* bv = lds + S.lds_bv;

    // Every unit ends with a barrier after the last reads of its LDS, so the
    // next unit may overwrite any of it before its first barrier.
    if (hb != cur_hb) {  // coefficient operands and biases of this stream's filter
      cur_hb = hb;
      const AOL_GLOBAL v4i* gh = (const AOL_GLOBAL v4i*)S.hfrag;
      const AOL_GLOBAL v4i* gv = (const AOL_GLOBAL v4i*)S.vfrag;
      for (int i = ctid; i < hb->nfrag * 64; i += NW * 64) ((v4i*)fh)[i] = gh[i];
      for (int i = ctid; i < vb->nfrag * 64; i += NW * 64) ((v4i*)fv)[i] = gv[i];
      if constexpr (ELEM == kU8) {
        for (int i = ctid; i < hb->nblk * 16; i += NW * 64) ((int*)bh)[i] = hb->bias[i];
        for (int i = ctid; i < vb->nblk * 16; i += NW * 64) ((int*)bv)[i] = vb->bias[i];
      }
      const AOL_GLOBAL uint32_t* gt = (const AOL_GLOBAL uint32_t*)S.vtab;
      for (int i = ctid; i < 2 * 64; i += NW * 64) ((uint32_t*)(lds + S.lds_vt))[i] = gt[i];
    }
    if constexpr (ELEM != kU8) {
      // float ring starts at zero so the zero taps of a block's padding never meet a NaN
      for (int i = ctid; i < (S.nbh * 16 * S.rpitch) / 16; i += NW * 64) {
        reinterpret_cast<v4i*>(zs)[i] = v4i{0, 0, 0, 0};
        reinterpret_cast<v4i*>(zs + S.zhalf)[i] = v4i{0, 0, 0, 0};
      }
    }
    // This wave's shares of the horizontal pass (a share takes blocks of one
    // position of the period): with loading-wave shares, the last NW of
    // LS * 8 + NW; without, one per compute wave, two when the filter has
    // more positions per period than there are compute waves. Then the
    // unit's vertical blocks (lane B: block B). (The second share is set up
    // unconditionally, with no blocks when unused: state set on one path
    // only would lose its uniformity to the compiler.)
    const int nv = LS > 0 ? LS * kBandLoadWaves + NW : hb->nblk > NW ? 2 * NW : NW;
    BandH<ELEM, split, KM, NBH> H;
    BandH<ELEM, split, KM, NBH, false> H2;  // (rarely used: operands read from LDS)
    H.setup(S, G, lds, LS > 0 ? (LS - 1) * kBandLoadWaves + wave : cw, nv, lane);
    if constexpr (LS == 0) H2.setup(S, G, lds, cw + NW, nv, lane);
    uint32_t vtbl = 0;  // lane B: vertical block B (read after the unit's first barrier)
    int vneed = 0;      // and the intermediate lines its window reaches
    const int vz = vb->zfrag;
    const uint8_t* fvl = fv + lane * 16;
    int B = 0;  // next vertical block
    int needB = 0;

    // ---- vertical blocks whose window lies in the first `have` intermediate lines
    auto vpass = [&](int have) {
      while (B < G.NBV && needB <= have) {
        const uint32_t t = __builtin_amdgcn_readlane(vtbl, B);
        const int c0 = (int)(t & 0xFFFFu), fb = (int)((t >> 16) & 0xFFu), lb = (int)((t >> 24) & 31u);
        const int nk = (int)(t >> 29);
        // this block's coefficient operands and ring offsets, for every column block
        v4i bf[KM], bfh[split ? KM : 1];
        int aoff[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const bool on = k < nk;
          const int f = on ? fb + k : vz;
          if constexpr (split) {
            bf[k] = *reinterpret_cast<const v4i*>(fvl + (2 * f) * 1024);
            bfh[k] = *reinterpret_cast<const v4i*>(fvl + (2 * f + 1) * 1024);
          } else {
            bf[k] = *reinterpret_cast<const v4i*>(fvl + f * 1024);
          }
          aoff[k] = ((c0 + ((on ? 4 * k : 0) + g) * E) % S.ring) * ES;  // ring bytes of the lane's chunk
        }
        const int bias = ELEM == kU8 ? *reinterpret_cast<const int*>(bv + lb * 64 + n * 4) : 0;
        const int orow = G.orow0 + 16 * B + n;
        // uniform: the block's 16 rows inside the plane, with rows 4- (rows_in)
        // or 2-element aligned (rows_in2)
        const bool rows_all = G.orow0 + 16 * B + 16 <= G.row_end;
        const bool rows_in = G.vec_out == 4 && rows_all;
        const bool rows_in2 = G.vec_out != 0 && rows_all;
        gdst_t rowp = G.dst + ((int64_t)orow * S.out_pitch + G.ocol0 + 4 * g) * (ELEM == kU8 ? 1 : 4);
        if constexpr (ELEM == kU8 && NB == 4) {
          // Integer outputs by pairs of adjacent column blocks: one swap of
          // lane-group halves (v_permlane16_swap) leaves each lane 8
          // consecutive bytes of one row, so one store covers 16 rows x 32
          // bytes instead of 16 rows x 16 bytes. Wave cw takes pairs cw,
          // cw + NW, cw + 2 NW, ..., two per iteration.
          const bool pitch8 = (S.out_pitch & 7) == 0;
          gdst_t rowq = G.dst + (int64_t)orow * S.out_pitch + G.ocol0 + 16 * (g & 1) + 8 * (g >> 1);
          for (int p0 = cw; 2 * p0 < G.nbh; p0 += 2 * NW) {
            v4i a[4][KM];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int cb = min(2 * (p0 + (j >> 1) * NW) + (j & 1), G.nbh - 1);
              const uint8_t* zr = zs + (16 * cb + n) * S.rpitch;
#pragma unroll
              for (int k = 0; k < KM; ++k) a[j][k] = *reinterpret_cast<const v4i*>(zr + aoff[k]);
            }
            v4i acc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = v4i{bias, bias, bias, bias};
#pragma unroll
            for (int k = 0; k < KM; ++k) {
              if (k > 0 && k >= nk) break;  // uniform
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], bf[k], acc[j], 0, 0, 0);
            }
            uint32_t y4[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) y4[j] = b_quant4(acc[j], 0);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int cbA = 2 * (p0 + q * NW);  // first block of the pair
              if (q > 0 && cbA >= G.nbh) break;
              const auto sw = __builtin_amdgcn_permlane16_swap(y4[2 * q], y4[2 * q + 1], false, false);
              // uniform: both blocks whole and inside the plane
              const bool pair_in = cbA + 1 < G.nbh && G.ocol0 + 16 * cbA + 32 <= G.col_end;
              if (rows_in && pitch8 && pair_in) {
                *(AOL_GLOBAL v2u*)(rowq + 16 * cbA) = v2u{(uint32_t)sw[0], (uint32_t)sw[1]};
              } else if (rows_in && pair_in) {
                *(AOL_GLOBAL uint32_t*)(rowq + 16 * cbA) = (uint32_t)sw[0];
                *(AOL_GLOBAL uint32_t*)(rowq + 16 * cbA + 4) = (uint32_t)sw[1];
              } else if (rows_in2 && pair_in) {
#pragma unroll
                for (int h = 0; h < 4; ++h)
                  *(AOL_GLOBAL uint16_t*)(rowq + 16 * cbA + 2 * h) = (uint16_t)((uint32_t)sw[h >> 1] >> (16 * (h & 1)));
              } else if (orow < G.row_end) {
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                  const int cb = cbA + jj;
                  const int col = G.ocol0 + 16 * cb + 4 * g;
                  if (cb < G.nbh) {
                    gdst_t op = rowp + 16 * cb;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                      if (col + i < G.col_end) op[i] = (uint8_t)(y4[2 * q + jj] >> (8 * i));
                  }
                }
              }
            }
          }
        } else {
          for (int cb0 = cw; cb0 < G.nbh; cb0 += NB * NW) {
            v4i a[NB][KM], al[NB][ELEM == kU8 ? 1 : KM];
  #pragma unroll
            for (int j = 0; j < NB; ++j) {
              const int cb = min(cb0 + j * NW, G.nbh - 1);
              const uint8_t* zr = zs + (16 * cb + n) * S.rpitch;
  #pragma unroll
              for (int k = 0; k < KM; ++k) {
                a[j][k] = *reinterpret_cast<const v4i*>(zr + aoff[k]);
                if constexpr (ELEM != kU8) al[j][k] = *reinterpret_cast<const v4i*>(zr + S.zhalf + aoff[k]);
              }
            }
            // All the products first, with no branch between them (a block
            // past the last repeats it; its result is not stored), so the
            // matrix-core latency of one block hides behind the others.
            v4i acc[NB], acch[split ? NB : 1];
            v4f accf[NB];
  #pragma unroll
            for (int j = 0; j < NB; ++j) {
              acc[j] = v4i{bias, bias, bias, bias};
              if constexpr (split) acch[j] = v4i{0, 0, 0, 0};
              accf[j] = v4f{0.f, 0.f, 0.f, 0.f};
            }
  #pragma unroll
            for (int k = 0; k < KM; ++k) {
              if (k > 0 && k >= nk) break;  // uniform
  #pragma unroll
              for (int j = 0; j < NB; ++j) {
                if constexpr (ELEM == kU8) {
                  acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], bf[k], acc[j], 0, 0, 0);
                  if constexpr (split) acch[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j][k], bfh[k], acch[j], 0, 0, 0);
                } else {
                  accf[j] = b_mfma16<ELEM>(a[j][k], bf[k], accf[j]);
                  accf[j] = b_mfma16<ELEM>(al[j][k], bf[k], accf[j]);
                }
              }
            }
  #pragma unroll
            for (int j = 0; j < NB; ++j) {
              const int cb = cb0 + j * NW;
              if (j > 0 && cb >= G.nbh) break;
              // uniform: the whole 16x16 output block inside the plane
              const bool cols_in = G.ocol0 + 16 * cb + 16 <= G.col_end;
              const bool inside = rows_in && cols_in, inside2 = rows_in2 && cols_in;
              const int col = G.ocol0 + 16 * cb + 4 * g;
              if constexpr (ELEM == kU8) {
                v4i r = acc[j];
                if constexpr (split) r = r + acch[j] * 128;
                const uint32_t y4 = b_quant4(r, 0);
                if (inside) {
                  *(AOL_GLOBAL uint32_t*)(rowp + 16 * cb) = y4;
                } else if (inside2) {
                  *(AOL_GLOBAL uint16_t*)(rowp + 16 * cb) = (uint16_t)y4;
                  *(AOL_GLOBAL uint16_t*)(rowp + 16 * cb + 2) = (uint16_t)(y4 >> 16);
                } else if (orow < G.row_end) {
                  gdst_t op = rowp + 16 * cb;
  #pragma unroll
                  for (int i = 0; i < 4; ++i)
                    if (col + i < G.col_end) op[i] = (uint8_t)(y4 >> (8 * i));
                }
              } else {
                if (inside) {
                  *(AOL_GLOBAL v4f*)(rowp + 64 * cb) = accf[j];
                } else if (inside2) {
                  *(AOL_GLOBAL v2f*)(rowp + 64 * cb) = v2f{accf[j][0], accf[j][1]};
                  *(AOL_GLOBAL v2f*)(rowp + 64 * cb + 8) = v2f{accf[j][2], accf[j][3]};
                } else if (orow < G.row_end) {
                  AOL_GLOBAL float* op = (AOL_GLOBAL float*)(rowp + 64 * cb);
  #pragma unroll
                  for (int i = 0; i < 4; ++i)
                    if (col + i < G.col_end) op[i] = accf[j][i];
                }
              }
            }
          }
        }
        ++B;
        needB = __builtin_amdgcn_readlane(vneed, min(B, 63));
      }
    };

    lds_barrier();  // step 0 staged, coefficients in place
    H.load_operands();
    if constexpr (LS == 0) H2.load_operands();
    {
      const uint32_t* vt = reinterpret_cast<const uint32_t*>(lds + S.lds_vt);
      vtbl = lane < G.NBV ? vt[lane] : 0u;
      vneed = lane < G.NBV ? min(G.Lz, (int)vt[64 + lane]) : 0;
      needB = __builtin_amdgcn_readlane(vneed, 0);
    }
    int zm = 0;     // ring line of step m's first intermediate line
    for (int m = 0; m < G.M; ++m) {
      // vertical blocks complete with step m-1's lines (the horizontal pass of
      // step m writes other ring lines meanwhile)
      vpass(min(G.Lz, 16 * m));
      H.run(zm, (t0 + m) & 1, g);  // this wave's shares of step m's horizontal pass
      if constexpr (LS == 0) H2.run(zm, (t0 + m) & 1, g);
      zm = zm + 16 == S.ring ? 0 : zm + 16;
      lds_barrier();  // step m's intermediate lines written, step m+1 staged
    }
    vpass(G.Lz);    // the rest of the unit's vertical blocks
    lds_barrier();  // the unit's LDS free
    t0 += G.M;
  }
}

template <int ELEM, int SLOTS, bool SPLIT, int KM, bool GATHER>
__global__ __launch_bounds__(kBandThreads) void k_band(BandLaunch L) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  band_body<ELEM, SLOTS, SPLIT, KM, GATHER>(L, lds);
}

// One launch of two parts of an integer batch on disjoint workgroups: the
// first A.ngroups workgroups run the streams whose taps fit int8, the others
// those whose taps are split (each part with its own kernel body, units and
// balanced schedule).
template <int SLOTS_A, int SLOTS_B, int KM>
__global__ __launch_bounds__(kBandThreads) void k_band_dual(BandLaunch A, BandLaunch B) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  if ((int)blockIdx.x < B.wg0) band_body<kU8, SLOTS_A, false, KM, false>(A, lds);
  else band_body<kU8, SLOTS_B, true, KM, false>(B, lds);
}

using BandFn = void (*)(BandLaunch);
using BandDualFn = void (*)(BandLaunch, BandLaunch);

template <int ELEM, bool SPLIT, int KM>
static BandFn band_pick_s(int slots) {
  if (slots <= 1) return k_band<ELEM, 1, SPLIT, KM, false>;
  if (slots <= 2) return k_band<ELEM, 2, SPLIT, KM, false>;
  if (slots <= 4) return k_band<ELEM, 4, SPLIT, KM, false>;
  return k_band<ELEM, 8, SPLIT, KM, false>;
}

// The gathering instance serves every slot and K-step count (the widest).
template <int ELEM, bool SPLIT>
static BandFn band_pick_k(int slots, int kmax, bool gather) {
  if (gather) return k_band<ELEM, kBandMaxSlots, SPLIT, kMaxK, true>;
  if (kmax <= 1) return band_pick_s<ELEM, SPLIT, 1>(slots);
  return kmax <= 2 ? band_pick_s<ELEM, SPLIT, 2>(slots) : band_pick_s<ELEM, SPLIT, 4>(slots);
}

static BandFn band_pick(int elem, int slots, bool split, int kmax, bool gather) {
  if (elem == kU8) return split ? band_pick_k<kU8, true>(slots, kmax, gather) : band_pick_k<kU8, false>(slots, kmax, gather);
  if (elem == kBF16) return band_pick_k<kBF16, false>(slots, kmax, gather);
  return band_pick_k<kFP16, false>(slots, kmax, gather);
}

hipError_t band_prepare(int elem, int slots, bool split, int kmax, size_t lds_bytes, int* wg_per_cu) {
  // both instances (whole chunks, gathering) are launchable with this LDS
  int wg[2] = {0, 0};
  for (int gather = 0; gather < 2; ++gather) {
    const void* f = (const void*)band_pick(elem, slots, split, kmax, gather != 0);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&wg[gather], f, kBandThreads, lds_bytes);
    if (e != hipSuccess) return e;
  }
  *wg_per_cu = wg[0] < wg[1] ? wg[0] : wg[1];
  return hipSuccess;
}

hipError_t band_launch(int elem, int slots, bool split, int kmax, bool gather, const BandLaunch& L, int grid,
                       size_t lds_bytes, hipStream_t stream) {
  BandLaunch La = L;
  La.wg0 = 0;
  La.ngroups = grid;
  hipLaunchKernelGGL(band_pick(elem, slots, split, kmax, gather), dim3(grid), dim3(kBandThreads), lds_bytes, stream, La);
  return hipGetLastError();
}

// Instances: staging slots 4 or 8 per part (fewer are served by 4), one or
// two K-steps.
template <int KM>
static BandDualFn band_dual_pick_k(int slots_a, int slots_b) {
  if (slots_a <= 4) return slots_b <= 4 ? k_band_dual<4, 4, KM> : k_band_dual<4, 8, KM>;
  return slots_b <= 4 ? k_band_dual<8, 4, KM> : k_band_dual<8, 8, KM>;
}

static BandDualFn band_dual_pick(int slots_a, int slots_b, int kmax) {
  return kmax <= 1 ? band_dual_pick_k<1>(slots_a, slots_b) : band_dual_pick_k<2>(slots_a, slots_b);
}

bool band_dual_supported(int slots_a, int slots_b, int kmax) {
  return slots_a <= 8 && slots_b <= 8 && kmax <= 2;
}

hipError_t band_dual_prepare(int slots_a, int slots_b, int kmax, size_t lds_bytes, int* wg_per_cu) {
  const void* f = (const void*)band_dual_pick(slots_a, slots_b, kmax);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg_per_cu, f, kBandThreads, lds_bytes);
}

hipError_t band_dual_launch(int slots_a, int slots_b, int kmax, const BandLaunch& A, int grid_a, const BandLaunch& B,
                            int grid_b, size_t lds_bytes, hipStream_t stream) {
  BandLaunch La = A, Lb = B;
  La.wg0 = 0;
  La.ngroups = grid_a;
  Lb.wg0 = grid_a;
  Lb.ngroups = grid_b;
  hipLaunchKernelGGL(band_dual_pick(slots_a, slots_b, kmax), dim3(grid_a + grid_b), dim3(kBandThreads), lds_bytes,
                     stream, La, Lb);
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
