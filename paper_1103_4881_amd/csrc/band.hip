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
  int r[SLOTS];    // line of the step
  int col[SLOTS];  // first element of the chunk, wrapped into the line
  int xo[SLOTS];   // LDS byte offset of the chunk in the staging lines

  __device__ __forceinline__ void setup(const BandStream& S, const BandUnitGeo& G, int ltid) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int idx = ltid + s * kBandLoadThreads;
      int rr = (int)__umulhi((uint32_t)idx, S.nch_magic);  // idx / nch
      int c = idx - rr * S.nch;
      // a lane past the last chunk loads and stores chunk 0 of line 15 again:
      // the same bytes to the same place, and no branch around the store,
      // which would leave its register's load outstanding on the other path
      if (rr >= 16) { rr = 15; c = 0; }
      xo[s] = rr * S.xpitch + c * 16;
      r[s] = rr;
      int cl = G.a0 + c * E;
      if (cl < 0 || cl >= S.w) cl = bpmod(cl, S.w);
      col[s] = cl;
    }
  }

  __device__ __forceinline__ gsrc_t line(const BandStream& S, const BandUnitGeo& G, int m, int s) const {
    const int l = min(16 * m + r[s], G.Lz - 1);
    int grow = G.zrow0 + l;
    if (grow < 0 || grow >= S.h) grow = bpmod(grow, S.h);
    return G.src + (int64_t)grow * S.in_pitch * ES;
  }

  // Whole chunks of a circular line (a wrapped chunk is another chunk).
  // Straight-line code with the same loads on every path, so the compiler's
  // count of loads in flight stays exact: rows are clamped and wrapped with
  // arithmetic, and a step past the unit loads its last line again.
  __device__ __forceinline__ void issue(v4i (&pre)[SLOTS], const BandStream& S, const BandUnitGeo& G, int m) const {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int grow = bpmod(G.zrow0 + min(16 * m + r[s], G.Lz - 1), S.h);
      pre[s] = *(const AOL_GLOBAL v4i*)(G.src + ((int64_t)grow * S.in_pitch + col[s]) * ES);
    }
  }

  // lines whose chunks are not whole chunks of the line: gathered element by
  // element with the wrap (a call, which waits for every load it issues)
  // and staged at once
  __device__ __forceinline__ void stage_gathered(const BandStream& S, const BandUnitGeo& G, int m, uint8_t* xs) const {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const v4i a = b_load_chunk_wrap<ES>(line(S, G, m, s), col[s], S.w);
      *reinterpret_cast<v4i*>(xs + xo[s]) = a;
    }
  }

  __device__ __forceinline__ void commit(const v4i (&pre)[SLOTS], uint8_t* xs) const {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) *reinterpret_cast<v4i*>(xs + xo[s]) = pre[s];
  }
};

// Loading waves of one unit: keep D steps of input lines in flight in
// registers and commit step m+1 into the staging lines while the compute
// waves run the vertical pass of step m. These waves issue no stores to
// memory, so their waits on loads count exactly (on gfx9 a wave with loads
// and stores outstanding can only wait for all of them).
template <int ELEM, int SLOTS>
__device__ __forceinline__ void band_feed_unit(const BandFeed<ELEM, SLOTS>& F, const BandStream& S,
                                               const BandUnitGeo& G, uint8_t* xs) {
  constexpr int D = BandDepth<SLOTS>::value;
  v4i pre[D][SLOTS];
#pragma unroll
  for (int k = 0; k < D; ++k) F.issue(pre[k], S, G, k);
  F.commit(pre[0], xs);
  F.issue(pre[0], S, G, D);
  lds_barrier();  // step 0 staged
  // Every iteration commits and re-issues one register set, so the loads in
  // flight at the loop head are the same sets in the same order on entry and
  // on the back edge. Steps past the unit stage its last line again into
  // staging lines nobody reads any more.
  // The loop runs whole groups of D steps, without an exit in between (an
  // exit path would reach the loop head with other loads in flight).
  int m0 = 0;
  for (; m0 + D <= G.M; m0 += D) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      lds_barrier();  // horizontal pass of step m0+k done with the staging lines
      const int j = (k + 1) % D;  // a constant once the loop is unrolled
      F.commit(pre[j], xs);
      F.issue(pre[j], S, G, m0 + k + 1 + D);
      lds_barrier();  // step m0+k+1 staged
    }
  }
#pragma unroll
  for (int k = 0; k + 1 < D; ++k) {
    if (m0 + k < G.M) {
      lds_barrier();
      F.commit(pre[(k + 1) % D], xs);
      lds_barrier();
    }
  }
  // nothing of this unit stays in flight into the next one
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// The same for lines that are gathered element by element: no prefetch.
template <int ELEM, int SLOTS>
__device__ __forceinline__ void band_feed_unit_gathered(const BandFeed<ELEM, SLOTS>& F, const BandStream& S,
                                                                  const BandUnitGeo& G, uint8_t* xs) {
  F.stage_gathered(S, G, 0, xs);
  lds_barrier();  // step 0 staged
  for (int m = 0; m < G.M; ++m) {
    lds_barrier();  // horizontal pass of step m done with the staging lines
    if (m + 1 < G.M) F.stage_gathered(S, G, m + 1, xs);
    lds_barrier();  // step m+1 staged
  }
}

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
  const cband_t hb = (cband_t)S.hb;
  const cband_t vb = (cband_t)S.vb;
  const AOL_CONST uint64_t* table = (const AOL_CONST uint64_t*)L.ptr_table;
  const uint64_t pin = table ? table[2 * S.ptr] : (uint64_t)L.ptrs[2 * S.ptr];
  const uint64_t pout = table ? table[2 * S.ptr + 1] : (uint64_t)L.ptrs[2 * S.ptr + 1];
  const int64_t fin = L.ptr_table ? 0 : L.fstride[2 * S.ptr];
  const int64_t fout = L.ptr_table ? 0 : L.fstride[2 * S.ptr + 1];
  G.src = (gsrc_t)pin + (int64_t)frame * fin * ES;
  G.dst = (gdst_t)pout + (int64_t)frame * fout * (ELEM == kU8 ? 1 : 4);
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

template <int ELEM, int SLOTS, bool SPLIT>
__global__ __launch_bounds__(kBandThreads) void k_band(BandLaunch L) {
  constexpr int ES = ELEM == kU8 ? 1 : 2;
  constexpr int E = 16 / ES;
  constexpr bool split = (ELEM == kU8) && SPLIT;
  constexpr int NW = (kBandThreads - kBandLoadThreads) / 64;  // compute waves
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool loader = wave < kBandLoadThreads / 64;
  const int cw = wave - kBandLoadThreads / 64;  // compute wave index
  const int ctid = tid - kBandLoadThreads;
  const int g = lane >> 4, n = lane & 15;

  // The two roles loop over the same units separately, so that the loading
  // waves' code never has a store in flight.
  if (loader) {
    for (int u = blockIdx.x; u < L.total_units; u += gridDim.x) {
      BandStream S;
      BandUnitGeo G;
      band_unit<ELEM>(L, u, S, G);
      uint8_t* xs = lds + S.lds_x;
      BandFeed<ELEM, SLOTS> F;
      F.setup(S, G, tid);
      if (G.vec_in) band_feed_unit<ELEM, SLOTS>(F, S, G, xs);
      else band_feed_unit_gathered<ELEM, SLOTS>(F, S, G, xs);
    }
    return;
  }

  cband_t cur_hb = nullptr;
  for (int u = blockIdx.x; u < L.total_units; u += gridDim.x) {
    BandStream S;
    BandUnitGeo G;
    band_unit<ELEM>(L, u, S, G);
    const cband_t hb = (cband_t)S.hb;
    const cband_t vb = (cband_t)S.vb;
    uint8_t* xs = lds + S.lds_x;
    uint8_t* zs = lds + S.lds_z;
    const v4i* fh = reinterpret_cast<const v4i*>(lds + S.lds_fh);
    const v4i* fv = reinterpret_cast<const v4i*>(lds + S.lds_fv);
    const int* bh = reinterpret_cast<const int*>(lds + S.lds_bh);
    const int* bv = reinterpret_cast<const int*>(lds + S.lds_bv);
    const int RM = S.ring - 1;

    // Every unit ends with a barrier after the last reads of its LDS, so the
    // next unit may overwrite any of it before its first barrier.
    if (hb != cur_hb) {  // coefficient operands and biases of this stream's filter
      cur_hb = hb;
      const AOL_GLOBAL v4i* gh = (const AOL_GLOBAL v4i*)S.hfrag;
      const AOL_GLOBAL v4i* gv = (const AOL_GLOBAL v4i*)S.vfrag;
      for (int i = ctid; i < hb->nfrag * 64; i += NW * 64) const_cast<v4i*>(fh)[i] = gh[i];
      for (int i = ctid; i < vb->nfrag * 64; i += NW * 64) const_cast<v4i*>(fv)[i] = gv[i];
      if constexpr (ELEM == kU8) {
        for (int i = ctid; i < hb->nblk * 16; i += NW * 64) const_cast<int*>(bh)[i] = hb->bias[i];
        for (int i = ctid; i < vb->nblk * 16; i += NW * 64) const_cast<int*>(bv)[i] = vb->bias[i];
      }
    }
    if constexpr (ELEM != kU8) {
      // float ring starts at zero so the zero taps of a block's padding never meet a NaN
      for (int i = ctid; i < (S.nbh * 16 * S.rpitch) / 16; i += NW * 64) {
        reinterpret_cast<v4i*>(zs)[i] = v4i{0, 0, 0, 0};
        reinterpret_cast<v4i*>(zs + S.zhalf)[i] = v4i{0, 0, 0, 0};
      }
    }
    lds_barrier();  // step 0 staged, coefficients in place

    int B = 0;  // next vertical block
    for (int m = 0; m < G.M; ++m) {
      // ---- horizontal pass: 16 intermediate lines of every 16-column block
      if constexpr (ELEM == kU8 && !split) {
        // two blocks per iteration: their LDS reads and MFMAs overlap
        for (int b0 = cw; b0 < G.nbh; b0 += 2 * NW) {
          const int b1 = b0 + NW;
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
      for (int b = cw; b < G.nbh; b += NW) {
        const int per = b / hb->nblk, lb = b - per * hb->nblk;
        const int c0 = hb->chunk0[lb] + per * (hb->q * 16 / E);  // a period is 16q elements
        const int nk = hb->nk[lb], fb = hb->frag[lb];
        const uint8_t* xr = xs + n * S.xpitch;
        if constexpr (ELEM == kU8) {
          v4i acc = {0, 0, 0, 0}, acch = {0, 0, 0, 0};
          for (int kb = 0; kb < nk; ++kb) {
            const v4i av = b_to_i8(*reinterpret_cast<const v4i*>(xr + (c0 + 4 * kb + g) * 16));
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fh[((fb + kb) * 2) * 64 + lane], acc, 0, 0, 0);
            acch = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, fh[((fb + kb) * 2 + 1) * 64 + lane], acch, 0, 0, 0);
          }
          acc = acc + acch * 128;
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
      // ---- vertical blocks whose window is complete
      const int have = min(G.Lz, 16 * (m + 1));
      while (B < G.NBV) {
        const int per = B / vb->nblk, lb = B - per * vb->nblk;
        const int need = min(G.Lz, vb->wend[lb] + 16 * per * vb->q);
        if (need > have) break;
        const int c0 = vb->chunk0[lb] + per * (vb->q * 16 / E);  // chunks of E intermediate lines
        const int nk = vb->nk[lb], fb = vb->frag[lb];
        const int orow = G.orow0 + 16 * B + n;
        for (int cb = cw; cb < G.nbh; cb += NW) {
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
              gdst_t op = G.dst + (int64_t)orow * S.out_pitch + col;
              if (G.vec_out && col + 4 <= G.col_end) {
                *(AOL_GLOBAL uint32_t*)op = y4;
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
              AOL_GLOBAL float* op = (AOL_GLOBAL float*)G.dst + (int64_t)orow * S.out_pitch + col;
              if (G.vec_out && col + 4 <= G.col_end) {
                *(AOL_GLOBAL v4f*)op = acc;
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
      lds_barrier();  // ring reads of this step done, step m+1 staged
    }
  }
}

using BandFn = void (*)(BandLaunch);

template <int ELEM, bool SPLIT>
static BandFn band_pick_s(int slots) {
  if (slots <= 1) return k_band<ELEM, 1, SPLIT>;
  if (slots <= 2) return k_band<ELEM, 2, SPLIT>;
  if (slots <= 4) return k_band<ELEM, 4, SPLIT>;
  return k_band<ELEM, 8, SPLIT>;
}

static BandFn band_pick(int elem, int slots, bool split) {
  if (elem == kU8) return split ? band_pick_s<kU8, true>(slots) : band_pick_s<kU8, false>(slots);
  if (elem == kBF16) return band_pick_s<kBF16, false>(slots);
  return band_pick_s<kFP16, false>(slots);
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
