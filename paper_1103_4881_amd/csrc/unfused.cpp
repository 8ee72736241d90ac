// Unfused downscaler: the horizontal and vertical filters as two kernels
// exchanging the intermediate frame through HBM (Sec. III-A: separate
// components connected by frame arrays), the counterpart of the fused
// kernel's on-chip intermediate. Same results as the fused path, bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "aolmi.h"
#include "common.h"
#include "plan.h"
#include "rowpass.h"

// Workspace of the allocation-free entry point: a static device array, one
// per GPU (each device holds its own copy, at its own address, for as long as
// the library is loaded). Its host-side name is not a device address: host
// code uses only the address hipGetSymbolAddress returns for the current
// device, resolved once per device at plan creation.
static __device__ __align__(256) uint8_t scratch[kStaticWorkBytes];

namespace aol {

static std::mutex g_scratch_mu;
static std::vector<uint8_t*> g_scratch_ptr;  // per device ordinal

aol_status static_workspace(uint8_t** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static workspace");
    g_scratch_ptr[dev] = (uint8_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return AOL_OK;
}

static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Kernel arguments of one pass over frames [f0, f0 + nf): horizontal (h) from
// the input planes into the workspace, vertical (!h) from the workspace into
// the output planes.
static void pass_args(const aol_plan* pl, bool h, int f0, int nf, const uint8_t* const* d_in, const int64_t* in_fs,
                      uint8_t* const* d_out, const int64_t* out_fs, uint8_t* work, RowPassArgs& a) {
  memset(&a, 0, sizeof a);
  const RowPassTables& t = h ? pl->uh : pl->uv;
  int tiles = 0;
  for (int i = 0; i < pl->n_planes; ++i) {
    const aol_plane_desc& d = pl->planes[i];
    RowPassPlane& P = a.pl[i];
    uint8_t* z = work + pl->uws_off[i];
    if (h) {
      P.in = d_in[i] + (int64_t)f0 * in_fs[i];
      P.in_pitch = d.in_pitch;
      P.in_fstride = in_fs[i];
      P.out = z;
      P.out_pitch = pl->uws_pitch[i];
      P.out_fstride = pl->uws_frame;
      P.rows = (int32_t)d.height;
      P.n = (int32_t)d.width;
      P.m = (int32_t)pl->mw[i];
      P.vec_in = (uintptr_t)P.in % 16 == 0 && d.in_pitch % 16 == 0 && (nf == 1 || in_fs[i] % 16 == 0);
      P.vec_out = 16;  // workspace: 256-byte aligned planes, 128-byte multiple pitches
    } else {
      P.in = z;
      P.in_pitch = pl->uws_pitch[i];
      P.in_fstride = pl->uws_frame;
      P.out = d_out[i] + (int64_t)f0 * out_fs[i];
      P.out_pitch = d.out_pitch;
      P.out_fstride = out_fs[i];
      P.rows = (int32_t)pl->mw[i];
      P.n = (int32_t)d.height;
      P.m = (int32_t)pl->mh[i];
      P.vec_in = 1;
      auto aligned = [&](int a) {
        return (uintptr_t)P.out % a == 0 && d.out_pitch % a == 0 && (nf == 1 || out_fs[i] % a == 0);
      };
      P.vec_out = aligned(16) ? 16 : aligned(4) ? 4 : 1;
    }
    P.nblocks = ceil_div(P.m, 16);
    P.row_tiles = ceil_div(P.rows, kRowPassRows);
    P.blk_tiles = ceil_div(P.nblocks, kRowPassBlocks);
    P.tile_base = tiles;
    tiles += P.row_tiles * P.blk_tiles;
  }
  a.n_planes = pl->n_planes;
  a.tiles_per_frame = tiles;
  a.x0 = t.x0;
  a.band = (const AxisBand*)t.d_band.ptr;
  a.frag = t.d_frag.ptr;
}

// Both passes over all frames, in chunks of frames whose intermediates fit
// work_bytes. Enqueue only.
aol_status run_unfused(aol_plan* pl, int32_t n_frames, const uint8_t* const* d_in, const int64_t* in_fs,
                       uint8_t* const* d_out, const int64_t* out_fs, uint8_t* work, int64_t work_bytes,
                       hipStream_t stream) {
  if (!pl) return fail(AOL_ERR_INVALID, "NULL plan");
  if (pl->elem != kU8) return fail(AOL_ERR_INVALID, "the unfused form is integer only (plan precision AOL_PREC_U8)");
  if (pl->uws_frame == 0) return fail(AOL_ERR_UNSUPPORTED, "these filters have no unfused form");
  if (n_frames < 0) return fail(AOL_ERR_INVALID, "n_frames < 0");
  if (n_frames == 0) return ok();
  if (!d_in || !d_out || !in_fs || !out_fs) return fail(AOL_ERR_INVALID, "NULL pointer array");
  if (!work) return fail(AOL_ERR_INVALID, "NULL workspace");
  if ((uintptr_t)work % 256) return fail(AOL_ERR_INVALID, "workspace not 256-byte aligned");
  for (int i = 0; i < pl->n_planes; ++i) {
    const aol_plane_desc& d = pl->planes[i];
    if (!d_in[i] || !d_out[i]) return fail(AOL_ERR_INVALID, "plane %d: NULL buffer", i);
    if (n_frames > 1 && (in_fs[i] < d.in_pitch * (d.height - 1) + d.width ||
                         out_fs[i] < d.out_pitch * (pl->mh[i] - 1) + pl->mw[i]))
      return fail(AOL_ERR_INVALID, "plane %d: frame stride smaller than a frame", i);
  }
  const int64_t per = std::min<int64_t>(work_bytes / pl->uws_frame, n_frames);
  if (per < 1)
    return fail(AOL_ERR_INVALID, "workspace of %lld bytes holds no frame (%lld bytes per frame)", (long long)work_bytes,
                (long long)pl->uws_frame);
  for (int f0 = 0; f0 < n_frames; f0 += (int)per) {
    const int nf = (int)std::min<int64_t>(per, n_frames - f0);
    for (int h = 1; h >= 0; --h) {
      RowPassArgs a;
      pass_args(pl, h != 0, f0, nf, d_in, in_fs, d_out, out_fs, work, a);
      const int64_t tiles = (int64_t)a.tiles_per_frame * nf;
      const int64_t grid = (tiles + 7) / 8 * 8;
      if (grid > INT_MAX) return fail(AOL_ERR_UNSUPPORTED, "too many tiles in one launch");
      a.total_tiles = (int32_t)tiles;
      const AxisBand& b = (h ? pl->uh : pl->uv).band;
      hipError_t e = rowpass_launch(b.split != 0, b.kmax, a, (int)grid, stream);
      if (e != hipSuccess) return hip_fail(e, h ? "horizontal pass launch" : "vertical pass launch");
    }
  }
  return ok();
}

}  // namespace aol

extern "C" {

aol_status aol_unfused_workspace_bytes(aol_plan* plan, int64_t* bytes_per_frame) {
  if (!plan || !bytes_per_frame) return fail(AOL_ERR_INVALID, "NULL argument");
  if (plan->elem != kU8) return fail(AOL_ERR_INVALID, "the unfused form is integer only (plan precision AOL_PREC_U8)");
  if (plan->uws_frame == 0) return fail(AOL_ERR_UNSUPPORTED, "these filters have no unfused form");
  *bytes_per_frame = plan->uws_frame;
  return ok();
}

aol_status aol_downscale_u8_unfused(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                                    const int64_t* in_frame_stride, uint8_t* const* d_out,
                                    const int64_t* out_frame_stride, void* d_work, int64_t work_bytes,
                                    hipStream_t stream) {
  return run_unfused(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, (uint8_t*)d_work, work_bytes,
                     stream);
}

aol_status aol_downscale_u8_unfused_static(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                                           const int64_t* in_frame_stride, uint8_t* const* d_out,
                                           const int64_t* out_frame_stride, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (plan->elem != kU8) return fail(AOL_ERR_INVALID, "the unfused form is integer only (plan precision AOL_PREC_U8)");
  if (plan->uws_frame == 0) return fail(AOL_ERR_UNSUPPORTED, "these filters have no unfused form");
  if (plan->uws_frame > kStaticWorkBytes)
    return fail(AOL_ERR_UNSUPPORTED, "one frame's intermediate (%lld bytes) exceeds the static workspace (%lld bytes)",
                (long long)plan->uws_frame, (long long)kStaticWorkBytes);
  if (!plan->uws_static) return fail(AOL_ERR_INVALID, "the plan has no static workspace address");
  return run_unfused(plan, n_frames, d_in, in_frame_stride, d_out, out_frame_stride, plan->uws_static,
                     kStaticWorkBytes, stream);
}

}  // extern "C"
