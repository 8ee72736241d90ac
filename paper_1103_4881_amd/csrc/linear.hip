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
// whose pattern crosses a border wraps each axis.
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

// One workgroup per row of the repetition space (every index but the last
// fixed); thread l takes the row's points l, l + 256, ... and advances its
// wrapped input and output base points by a constant per step.
template <int NOUT>
__global__ __launch_bounds__(kLinThreads) void k_linear(LinearArgs a) {
  const int last = a.rr - 1;
  const int lane0 = threadIdx.x;
  if (lane0 >= a.R[last]) return;  // no barrier in this kernel
  // the row's repetition indices (uniform)
  int r[kLinRank] = {0, 0, 0, 0};
  {
    uint32_t row = blockIdx.x;
#pragma unroll
    for (int k = kLinRank - 1; k >= 0; --k) {
      if (k < last) {
        r[k] = (int)(row % (uint32_t)a.R[k]);
        row /= (uint32_t)a.R[k];
      }
    }
    r[last] = lane0;
  }
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

  for (int rl = lane0; rl < a.R[last]; rl += kLinThreads) {
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

}  // namespace aol
