// Host-to-host frame pipeline around a downscale plan: the transfers the
// paper measures (Sec. IV: host<->device copies dominate the generated
// application's time; its tuning removes redundant ones) organised as three
// overlapping stages. Groups of frames go host -> device on one copy stream,
// through the fused kernel on the caller's stream, and device -> host on a
// second copy stream; a ring of device slots lets the copies of one group run
// while another is filtered. Events order the stages and time them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "aolmi.h"
#include "common.h"
#include "plan.h"

using namespace aol;

struct aol_pipeline {
  aol_plan* plan = nullptr;
  int batch = 1, depth = 1;
  int n_planes = 0;
  int64_t in_bytes[kMaxPlanes] = {}, out_bytes[kMaxPlanes] = {};   // extent of one frame (bytes)
  int64_t din_fs[kMaxPlanes] = {}, dout_fs[kMaxPlanes] = {};       // device frame strides (bytes)
  std::vector<DeviceBuf> din, dout;                                // [slot * n_planes + plane]
  hipStream_t h2d = nullptr, d2h = nullptr;
  // per slot: h2d start/end, kernel start/end, d2h start/end
  std::vector<hipEvent_t> ev;
  hipEvent_t ev_first = nullptr, ev_last = nullptr;
  ~aol_pipeline() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (ev_first) (void)hipEventDestroy(ev_first);
    if (ev_last) (void)hipEventDestroy(ev_last);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
  }
};

namespace {

enum { kH2D0, kH2D1, kK0, kK1, kD2H0, kD2H1, kEvPerSlot };

hipEvent_t& slot_ev(aol_pipeline* pp, int slot, int which) { return pp->ev[(size_t)slot * kEvPerSlot + which]; }

double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
}

// Waits for the group in `slot` and adds its stage times.
aol_status retire(aol_pipeline* pp, int slot, aol_pipeline_stats* st) {
  hipError_t e = hipEventSynchronize(slot_ev(pp, slot, kD2H1));
  if (e != hipSuccess) return hip_fail(e, "waiting for a group's device-to-host copy");
  st->h2d_ms += elapsed(slot_ev(pp, slot, kH2D0), slot_ev(pp, slot, kH2D1));
  st->kernel_ms += elapsed(slot_ev(pp, slot, kK0), slot_ev(pp, slot, kK1));
  st->d2h_ms += elapsed(slot_ev(pp, slot, kD2H0), slot_ev(pp, slot, kD2H1));
  return AOL_OK;
}

}  // namespace

extern "C" {

aol_status aol_pipeline_create(aol_plan* plan, int32_t batch_frames, int32_t depth, aol_pipeline** out) {
  if (!out) return fail(AOL_ERR_INVALID, "NULL pipeline output");
  *out = nullptr;
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (plan->elem != kU8) return fail(AOL_ERR_INVALID, "pipelines run integer plans (AOL_PREC_U8)");
  if (batch_frames < 1 || depth < 1 || depth > 64) return fail(AOL_ERR_INVALID, "batch_frames >= 1, 1 <= depth <= 64");
  aol_pipeline* pp = new (std::nothrow) aol_pipeline();
  if (!pp) return fail(AOL_ERR_NOMEM, "pipeline allocation");
  pp->plan = plan;
  pp->batch = batch_frames;
  pp->depth = depth;
  pp->n_planes = plan->n_planes;
  for (int j = 0; j < plan->n_planes; ++j) {
    const aol_plane_desc& d = plan->planes[j];
    pp->in_bytes[j] = d.in_pitch * (d.height - 1) + d.width;
    pp->out_bytes[j] = d.out_pitch * (plan->mh[j] - 1) + plan->mw[j];
    pp->din_fs[j] = (d.in_pitch * d.height + 255) / 256 * 256;
    pp->dout_fs[j] = (d.out_pitch * plan->mh[j] + 255) / 256 * 256;
  }
  pp->din.resize((size_t)depth * plan->n_planes);
  pp->dout.resize((size_t)depth * plan->n_planes);
  aol_status st = AOL_OK;
  for (int s = 0; s < depth && !st; ++s)
    for (int j = 0; j < plan->n_planes && !st; ++j) {
      st = pp->din[(size_t)s * plan->n_planes + j].alloc((size_t)pp->din_fs[j] * batch_frames);
      if (!st) st = pp->dout[(size_t)s * plan->n_planes + j].alloc((size_t)pp->dout_fs[j] * batch_frames);
    }
  hipError_t e = hipSuccess;
  if (!st && (e = hipStreamCreateWithFlags(&pp->h2d, hipStreamNonBlocking)) != hipSuccess) st = hip_fail(e, "copy stream");
  if (!st && (e = hipStreamCreateWithFlags(&pp->d2h, hipStreamNonBlocking)) != hipSuccess) st = hip_fail(e, "copy stream");
  pp->ev.assign((size_t)depth * kEvPerSlot, nullptr);
  for (size_t i = 0; i < pp->ev.size() && !st; ++i)
    if ((e = hipEventCreate(&pp->ev[i])) != hipSuccess) st = hip_fail(e, "hipEventCreate");
  if (!st && (e = hipEventCreate(&pp->ev_first)) != hipSuccess) st = hip_fail(e, "hipEventCreate");
  if (!st && (e = hipEventCreate(&pp->ev_last)) != hipSuccess) st = hip_fail(e, "hipEventCreate");
  if (st) {
    delete pp;
    return st;
  }
  *out = pp;
  return ok();
}

aol_status aol_pipeline_destroy(aol_pipeline* pp) {
  if (pp) {
    (void)hipStreamSynchronize(pp->h2d);
    (void)hipStreamSynchronize(pp->d2h);
  }
  delete pp;
  return ok();
}

aol_status aol_pipeline_run_u8(aol_pipeline* pp, int32_t n_frames, const uint8_t* const* h_in,
                               const int64_t* in_frame_stride, uint8_t* const* h_out, const int64_t* out_frame_stride,
                               hipStream_t stream, aol_pipeline_stats* stats) {
  if (!pp) return fail(AOL_ERR_INVALID, "NULL pipeline");
  if (n_frames < 0) return fail(AOL_ERR_INVALID, "n_frames < 0");
  if (!h_in || !h_out || !in_frame_stride || !out_frame_stride) return fail(AOL_ERR_INVALID, "NULL pointer array");
  for (int j = 0; j < pp->n_planes; ++j) {
    if (n_frames > 0 && (!h_in[j] || !h_out[j])) return fail(AOL_ERR_INVALID, "plane %d: NULL host buffer", j);
    if (n_frames > 1 && (in_frame_stride[j] < pp->in_bytes[j] || out_frame_stride[j] < pp->out_bytes[j]))
      return fail(AOL_ERR_INVALID, "plane %d: frame stride smaller than a frame", j);
  }
  aol_pipeline_stats st;
  memset(&st, 0, sizeof st);
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e;
  if ((e = hipEventRecord(pp->ev_first, pp->h2d)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  const int groups = (n_frames + pp->batch - 1) / pp->batch;
  const uint8_t* din[kMaxPlanes];
  uint8_t* dout[kMaxPlanes];
  int64_t fin[kMaxPlanes], fout[kMaxPlanes];
  for (int b = 0; b < groups; ++b) {
    const int s = b % pp->depth;
    const int f0 = b * pp->batch, nb = std::min(pp->batch, n_frames - f0);
    if (b >= pp->depth) {  // the slot's previous group must be back on the host
      aol_status r = retire(pp, s, &st);
      if (r) return r;
    }
    if ((e = hipEventRecord(slot_ev(pp, s, kH2D0), pp->h2d)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int j = 0; j < pp->n_planes; ++j) {
      uint8_t* d = (uint8_t*)pp->din[(size_t)s * pp->n_planes + j].ptr;
      e = hipMemcpy2DAsync(d, (size_t)pp->din_fs[j], h_in[j] + (int64_t)f0 * in_frame_stride[j],
                           (size_t)std::max<int64_t>(in_frame_stride[j], pp->in_bytes[j]), (size_t)pp->in_bytes[j],
                           (size_t)nb, hipMemcpyHostToDevice, pp->h2d);
      if (e != hipSuccess) return hip_fail(e, "host-to-device copy");
      din[j] = d;
      dout[j] = (uint8_t*)pp->dout[(size_t)s * pp->n_planes + j].ptr;
      fin[j] = pp->din_fs[j];
      fout[j] = pp->dout_fs[j];
    }
    if ((e = hipEventRecord(slot_ev(pp, s, kH2D1), pp->h2d)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(stream, slot_ev(pp, s, kH2D1), 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    if ((e = hipEventRecord(slot_ev(pp, s, kK0), stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    aol_status r = aol_downscale_u8(pp->plan, nb, din, fin, dout, fout, stream);
    if (r) return r;
    if ((e = hipEventRecord(slot_ev(pp, s, kK1), stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(pp->d2h, slot_ev(pp, s, kK1), 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    if ((e = hipEventRecord(slot_ev(pp, s, kD2H0), pp->d2h)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int j = 0; j < pp->n_planes; ++j) {
      e = hipMemcpy2DAsync(h_out[j] + (int64_t)f0 * out_frame_stride[j],
                           (size_t)std::max<int64_t>(out_frame_stride[j], pp->out_bytes[j]), dout[j],
                           (size_t)pp->dout_fs[j], (size_t)pp->out_bytes[j], (size_t)nb, hipMemcpyDeviceToHost, pp->d2h);
      if (e != hipSuccess) return hip_fail(e, "device-to-host copy");
    }
    if ((e = hipEventRecord(slot_ev(pp, s, kD2H1), pp->d2h)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  for (int b = std::max(0, groups - pp->depth); b < groups; ++b) {
    aol_status r = retire(pp, b % pp->depth, &st);
    if (r) return r;
  }
  if ((e = hipEventRecord(pp->ev_last, pp->d2h)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = hipEventSynchronize(pp->ev_last)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  st.span_ms = groups ? elapsed(pp->ev_first, pp->ev_last) : 0.0;
  st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  st.groups = groups;
  st.frames = n_frames;
  for (int j = 0; j < pp->n_planes; ++j) {
    st.h2d_bytes += (int64_t)n_frames * pp->in_bytes[j];
    st.d2h_bytes += (int64_t)n_frames * pp->out_bytes[j];
  }
  if (stats) *stats = st;
  return ok();
}

}  // extern "C"
