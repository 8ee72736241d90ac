// Array-OL repetition with a linear integer elementary task (uint8 arrays),
// for gfx950.
//
// Sec. III: the application reads 24-bit RGB frames, filters their colour
// components and composes the output frame from the colour-space results;
// Sec. III-A and its tiler footnote: each step is a repetitive task whose
// input tiler cuts pattern element i of repetition r out of A at
// (o + P.r + F.i) mod S and whose output tiler writes result element j to B
// at (o' + P'.r + F'.j) mod S'. Here the elementary task is linear with
// integer weights:
//
//   y[j] = clamp(floor((sum_i W[j][i] x[i] + bias[j] + 128) / 256), 0, 255)
//
// which covers interleaved-RGB <-> planar colour conversions (3 -> 3),
// non-separable 2-D filters with several outputs per repetition (a 2-D
// polyphase downscale: span x span -> p x p) and box filters.
//
// Threads run along the last repetition dimension. The pattern offsets and
// weights are the same for every thread and come through scalar loads;
// pairs of pattern elements are multiplied
// with v_dot2_i32_i16 (two exact 16-bit products per instruction into an
// int32 accumulator, exact under the host's bound on sum |W| * 255).
// Patterns that stay inside the array use constant flat offsets; a point
// whose pattern crosses a border wraps each axis. For small patterns a staged
// form reads each chunk of a row's input from LDS, loaded with 16-byte loads,
// and stores dense output ranges from LDS the same way (byte-wide global
// accesses were its limit).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "linear.h"

namespace aol {

namespace {

typedef short v2s __attribute__((ext_vector_type(2)));
#define LIN_CONST __attribute__((address_space(4)))
typedef const LIN_CONST int32_t* ctab_t;
typedef const __attribute__((address_space(1))) uint8_t* lin_in_t;
typedef __attribute__((address_space(1))) uint8_t* lin_out_t;

}  // namespace

// Points xb + threadIdx.x, + kLinThreads, ... below xe of the repetition
// row r (every index but the last), point by point: each thread advances its
// wrapped input and output base points by a constant per step; a point whose
// pattern stays inside the array uses constant flat offsets, one that crosses
// a border wraps each axis.
template <int NOUT>
__device__ __forceinline__ void linear_points(const LinearArgs& a, const int (&r0)[kLinRank], int xb, int xe,
                                              int rot = 0) {
  const int last = a.rr - 1;
  int r[kLinRank];
#pragma unroll
  for (int k = 0; k < kLinRank; ++k) r[k] = r0[k];
  r[last] = xb + (int)threadIdx.x + rot;  // rot: only with xb = 0 and one point per thread
  if (r[last] >= a.R[last]) r[last] -= a.R[last];
  // wrapped base points of the thread's first point, input and output
  int b[kLinRank] = {0, 0, 0, 0}, ob[kLinRank] = {0, 0, 0, 0};
#pragma unroll
  for (int d = 0; d < kLinRank; ++d) {
    if (d < a.ra) {
      int64_t v = a.o[d];
#pragma unroll
      for (int k = 0; k < kLinRank; ++k)
        if (k < a.rr) v += (int64_t)a.P[d][k] * r[k];
      b[d] = (int)(v % a.S[d]);
    }
    if (d < a.ro) {
      int64_t v = a.oo[d];
#pragma unroll
      for (int k = 0; k < kLinRank; ++k)
        if (k < a.rr) v += (int64_t)a.Po[d][k] * r[k];
      ob[d] = (int)(v % a.So[d]);
    }
  }
  const ctab_t tab = (ctab_t)a.tab;
  const ctab_t ioff = tab;
  const ctab_t ifd = tab + a.t_ifd;
  const ctab_t wpair = tab + a.t_w;
  const ctab_t ooff = tab + a.t_ooff;
  const ctab_t ofd = tab + a.t_ofd;
  const int n2 = 2 * a.n_pairs;
  const lin_in_t in = (lin_in_t)a.in;
  const lin_out_t out = (lin_out_t)a.out;

  for (int rl = xb + (int)threadIdx.x; rl < xe; rl += kLinThreads) {
    bool inside = true, oinside = true;
    int flat = 0, oflat = 0;
#pragma unroll
    for (int d = 0; d < kLinRank; ++d) {
      if (d < a.ra) {
        inside = inside && b[d] + a.lo[d] >= 0 && b[d] + a.hi[d] < a.S[d];
        flat += b[d] * a.st[d];
      }
      if (d < a.ro) {
        oinside = oinside && ob[d] + a.olo[d] >= 0 && ob[d] + a.ohi[d] < a.So[d];
        oflat += ob[d] * a.sto[d];
      }
    }
    auto wrapped = [&](int i) -> uint32_t {
      int f = 0;
#pragma unroll
      for (int d = 0; d < kLinRank; ++d) {
        if (d < a.ra) {
          int c = b[d] + ifd[d * n2 + i];  // both in [0, S): one subtraction wraps
          if (c >= a.S[d]) c -= a.S[d];
          f += c * a.st[d];
        }
      }
      return in[f];
    };
    int acc[NOUT];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) acc[j] = tab[a.t_bias + j];
    auto madd = [&](int k, uint32_t x) {
      const v2s xv = __builtin_bit_cast(v2s, x);
#pragma unroll
      for (int j = 0; j < NOUT; ++j)
        acc[j] = __builtin_amdgcn_sdot2(xv, __builtin_bit_cast(v2s, wpair[k * NOUT + j]), acc[j], false);
    };
    if (inside) {  // the usual case: constant flat offsets, four pairs of loads in flight
      int k = 0;
      for (; k + 4 <= a.n_pairs; k += 4) {
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = in[flat + ioff[2 * (k + u)]] | ((uint32_t)in[flat + ioff[2 * (k + u) + 1]] << 16);
#pragma unroll
        for (int u = 0; u < 4; ++u) madd(k + u, x[u]);
      }
      for (; k < a.n_pairs; ++k) madd(k, in[flat + ioff[2 * k]] | ((uint32_t)in[flat + ioff[2 * k + 1]] << 16));
    } else {
      for (int k = 0; k < a.n_pairs; ++k) madd(k, wrapped(2 * k) | (wrapped(2 * k + 1) << 16));
    }
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
      if (j >= a.n_out) continue;  // uniform
      int f = oflat + ooff[j];
      if (!oinside) {
        f = 0;
#pragma unroll
        for (int d = 0; d < kLinRank; ++d) {
          if (d < a.ro) {
            int c = ob[d] + ofd[d * NOUT + j];
            if (c >= a.So[d]) c -= a.So[d];
            f += c * a.sto[d];
          }
        }
      }
      out[f] = (uint8_t)min(max(acc[j] >> 8, 0), 255);  // arithmetic shift: floor division by 256
    }
    // next point of the thread along the last repetition dimension
#pragma unroll
    for (int d = 0; d < kLinRank; ++d) {
      if (d < a.ra) {
        b[d] += a.inc[d];
        if (b[d] >= a.S[d]) b[d] -= a.S[d];
      }
      if (d < a.ro) {
        ob[d] += a.oinc[d];
        if (ob[d] >= a.So[d]) ob[d] -= a.So[d];
      }
    }
  }
}

// the repetition row of workgroup-row index `row` (every index but the last)
__device__ __forceinline__ void linear_row(const LinearArgs& a, uint32_t row, int (&r)[kLinRank]) {
  const int last = a.rr - 1;
#pragma unroll
  for (int k = kLinRank - 1; k >= 0; --k) {
    r[k] = 0;
    if (k < last) {
      r[k] = (int)(row % (uint32_t)a.R[k]);
      row /= (uint32_t)a.R[k];
    }
  }
}

// floor(n / d) for n, d < 2^31 from m = floor(2^32 / d) + 1 (the product's
// high word is the quotient or one more)
__device__ __forceinline__ uint32_t lin_div(uint32_t n, uint32_t d, uint32_t m) {
  if (d == 1) return n;  // m would be 2^32 + 1
  const uint32_t q = __umulhi(n, m);
  return q * d > n ? q - 1 : q;
}

// One workgroup per row of the repetition space; thread l takes the row's
// points l, l + 256, ...
template <int NOUT>
__global__ __launch_bounds__(kLinThreads) void k_linear(LinearArgs a) {
  int r[kLinRank];
  linear_row(a, blockIdx.x, r);
  linear_points<NOUT>(a, r, 0, a.R[a.rr - 1], a.rot);  // no barrier in this kernel
}

// The staged form (one workgroup per chunk of C = kLinThreads * ppt points of
// a row; see LinearStage). A chunk whose points all keep their whole input
// and output patterns inside the arrays, with no coordinate wrapping between
// its first and last point (a uniform test of the two ends per axis), reads
// its input ranges from LDS and writes dense output ranges through LDS; any
// other chunk runs point by point. Same arithmetic either way.
template <int NOUT>
__global__ __launch_bounds__(kLinThreads) void k_linear_staged(LinearArgs a, LinearStage st) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  typedef int v4i __attribute__((ext_vector_type(4)));
  const int last = a.rr - 1;
  const int tid = threadIdx.x;
  const uint32_t rowi = lin_div(blockIdx.x, (uint32_t)st.chunks, st.mg_R[last]);
  const int chunk = (int)(blockIdx.x - rowi * (uint32_t)st.chunks);
  const int C = kLinThreads * st.ppt;
  const int x0 = chunk * C;
  const int npts = min(C, a.R[last] - x0);  // uniform, >= 1
  const ctab_t tab = (ctab_t)a.tab;
  // the chunk's flat input and output positions of its first point, or -1:
  // not clean (computed on the host)
  const int flat0 = tab[st.cq + 2 * blockIdx.x], oflat0 = tab[st.cq + 2 * blockIdx.x + 1];
  const bool clean = flat0 >= 0;
  if (!clean) {  // uniform
    int r[kLinRank] = {0, 0, 0, 0};
    uint32_t row = rowi;
#pragma unroll
    for (int k = kLinRank - 1; k >= 0; --k) {
      if (k < last) {
        const uint32_t q = lin_div(row, (uint32_t)a.R[k], st.mg_R[k]);
        r[k] = (int)(row - q * (uint32_t)a.R[k]);
        row = q;
      }
    }
    linear_points<NOUT>(a, r, x0, x0 + npts);
    return;
  }
  const lin_in_t in = (lin_in_t)a.in;
  const lin_out_t out = (lin_out_t)a.out;
  const ctab_t grp = tab + st.t_grp;
  const ctab_t wpair = tab + a.t_w;
  // ---- the chunk's input ranges into LDS, 16-byte chunks aligned as in
  // memory: the byte at flat position F of group g sits at LDS gl[g] - A_g + F,
  // A_g the group's first position rounded down to 16 (every position the
  // chunk reads lies inside the array)
#pragma unroll
  for (int g = 0; g < kLinGroups; ++g) {
    if (g < st.ng) {
      const int start = flat0 + st.gb[g];
      const int end = start + (npts - 1) * st.P + st.gs[g];
      const int A = start & ~15;
      const int nch = (end - A + 15) >> 4;
      for (int c = tid; c < nch; c += kLinThreads) {
        const int F = A + 16 * c;
        v4i v;
        if ((int64_t)F + 16 <= st.n_in) {
          v = *(const __attribute__((address_space(1))) v4i*)(in + F);
        } else {  // the array's last chunk: its bytes only
          uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (F + q < st.n_in) w[q >> 2] |= (uint32_t)in[F + q] << (8 * (q & 3));
          v = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
        }
        *reinterpret_cast<v4i*>(lds + st.gl[g] + 16 * c) = v;
      }
    }
  }
  // ---- per element, its LDS position for the chunk's first point: etab[e]
  // (inputs), otab[j] (outputs staged in LDS) or the output's flat position
  int* etab = reinterpret_cast<int*>(lds);
  int* otab = etab + 2 * a.n_pairs;
  for (int e = tid; e < 2 * a.n_pairs + NOUT; e += kLinThreads) {
    if (e < 2 * a.n_pairs) {
      const int g = tab[st.t_eg + e];
      etab[e] = grp[4 * g + 1] - ((flat0 + grp[4 * g]) & ~15) + flat0 + tab[e];
    } else {
      const int j = e - 2 * a.n_pairs;
      const int g = tab[st.t_og + j];
      otab[j] = st.ngo > 0 ? grp[4 * g + 3] - ((oflat0 + grp[4 * g + 2]) & ~15) + oflat0 + tab[a.t_ooff + j]
                           : oflat0 + tab[a.t_ooff + j];
    }
  }
  __syncthreads();
  // ---- the points: point x0 + i reads etab[e] + i * P (one range: the
  // range's LDS base + ioff[e] + i * P), writes otab[j] + i * Po. A pass
  // takes PP points per thread (i, i + 256, ...), so each pair's offsets and
  // weights (scalar loads) serve PP points; a point past the chunk reads
  // position 0 and writes nothing.
  constexpr int PP = NOUT <= 2 ? 8 : NOUT <= 4 ? 4 : NOUT <= 8 ? 2 : 1;
  const int in_base1 = st.gl[0] - ((flat0 + st.gb[0]) & ~15) + flat0;
  for (int i0 = tid; i0 < npts; i0 += PP * kLinThreads) {
    int di[PP];
    bool ok[PP];
#pragma unroll
    for (int p = 0; p < PP; ++p) {
      const int i = i0 + p * kLinThreads;
      ok[p] = i < npts;
      di[p] = ok[p] ? i * st.P : 0;
    }
    int acc[PP][NOUT];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) {
      const int bj = tab[a.t_bias + j];
#pragma unroll
      for (int p = 0; p < PP; ++p) acc[p][j] = bj;
    }
    auto madd = [&](int k, const uint32_t (&x)[PP]) {
#pragma unroll
      for (int j = 0; j < NOUT; ++j) {
        const v2s w = __builtin_bit_cast(v2s, wpair[k * NOUT + j]);
#pragma unroll
        for (int p = 0; p < PP; ++p) acc[p][j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(v2s, x[p]), w, acc[p][j], false);
      }
    };
    for (int k = 0; k < a.n_pairs; ++k) {
      int e0, e1;
      if (st.ng == 1) {  // uniform: one range, the element offsets straight from the table
        e0 = in_base1 + tab[2 * k];
        e1 = in_base1 + tab[2 * k + 1];
      } else {
        const int2 e = reinterpret_cast<const int2*>(etab)[k];  // the same for every lane
        e0 = e.x;
        e1 = e.y;
      }
      uint32_t x[PP];
#pragma unroll
      for (int p = 0; p < PP; ++p) x[p] = (uint32_t)lds[e0 + di[p]] | ((uint32_t)lds[e1 + di[p]] << 16);
      madd(k, x);
    }
#pragma unroll
    for (int p = 0; p < PP; ++p) {
      if (!ok[p]) continue;
      const int dout = (i0 + p * kLinThreads) * st.Po;
#pragma unroll
      for (int j = 0; j < NOUT; ++j) {
        if (j >= a.n_out) continue;  // uniform
        const uint8_t y = (uint8_t)min(max(acc[p][j] >> 8, 0), 255);
        if (st.ngo > 0) lds[otab[j] + dout] = y;
        else out[otab[j] + dout] = y;
      }
    }
  }
  if (st.ngo == 0) return;  // uniform
  __syncthreads();
  // ---- the chunk's output ranges, whole aligned 16-byte chunks where they lie inside
#pragma unroll
  for (int g = 0; g < kLinGroups; ++g) {
    if (g < st.ngo) {
      const int S0 = oflat0 + st.ob[g], E0 = S0 + npts * st.Po;
      const int OA = S0 & ~15;
      const int nch = (E0 - OA + 15) >> 4;
      for (int c = tid; c < nch; c += kLinThreads) {
        const int F = OA + 16 * c;
        const uint8_t* src = lds + st.ol[g] + 16 * c;
        if (F >= S0 && F + 16 <= E0) {
          *(__attribute__((address_space(1))) v4i*)(out + F) = *reinterpret_cast<const v4i*>(src);
        } else {
          for (int q = max(F, S0); q < min(F + 16, E0); ++q) out[q] = src[q - F];
        }
      }
    }
  }
}

hipError_t linear_launch(int nout, const LinearArgs& a, hipStream_t stream) {
  const int64_t blocks = a.nrep / a.R[a.rr - 1];  // rows of the repetition space
  const dim3 grid((unsigned)blocks), block(kLinThreads);
  switch (nout) {
    case 1: hipLaunchKernelGGL(k_linear<1>, grid, block, 0, stream, a); break;
    case 2: hipLaunchKernelGGL(k_linear<2>, grid, block, 0, stream, a); break;
    case 3: hipLaunchKernelGGL(k_linear<3>, grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL(k_linear<4>, grid, block, 0, stream, a); break;
    case 6: hipLaunchKernelGGL(k_linear<6>, grid, block, 0, stream, a); break;
    case 8: hipLaunchKernelGGL(k_linear<8>, grid, block, 0, stream, a); break;
    case 9: hipLaunchKernelGGL(k_linear<9>, grid, block, 0, stream, a); break;
    case 12: hipLaunchKernelGGL(k_linear<12>, grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL(k_linear<16>, grid, block, 0, stream, a); break;
  }
  return hipGetLastError();
}

template <int NOUT>
static void staged_launch(const LinearArgs& a, const LinearStage& st, dim3 grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_linear_staged<NOUT>, grid, dim3(kLinThreads), (size_t)st.lds_bytes, stream, a, st);
}

hipError_t linear_staged_launch(int nout, const LinearArgs& a, const LinearStage& st, hipStream_t stream) {
  const int64_t rows = a.nrep / a.R[a.rr - 1];
  const dim3 grid((unsigned)(rows * st.chunks));
  switch (nout) {
    case 1: staged_launch<1>(a, st, grid, stream); break;
    case 2: staged_launch<2>(a, st, grid, stream); break;
    case 3: staged_launch<3>(a, st, grid, stream); break;
    case 4: staged_launch<4>(a, st, grid, stream); break;
    case 6: staged_launch<6>(a, st, grid, stream); break;
    case 8: staged_launch<8>(a, st, grid, stream); break;
    case 9: staged_launch<9>(a, st, grid, stream); break;
    case 12: staged_launch<12>(a, st, grid, stream); break;
    default: staged_launch<16>(a, st, grid, stream); break;
  }
  return hipGetLastError();
}

}  // namespace aol
