// The downscale plan object (shared by the fused and unfused entry points).
#pragma once
#include <string>
#include <vector>

#include "aol_internal.h"
#include "aolmi.h"
#include "band_host.h"
#include "common.h"

namespace aol {

// One axis of the unfused form: the period band of a row pass (16-byte
// chunk aligned) and its coefficient operands.
struct RowPassTables {
  AxisBand band{};
  int32_t x0 = 0;  // element of the period window's position 0, relative to 16*q*period
  DeviceBuf d_band, d_frag;
};

aol_status build_rowpass_tables(const FilterHost& f, RowPassTables& out, const char* name);

// Bytes of the static workspace of aol_downscale_u8_unfused_static.
constexpr int64_t kStaticWorkBytes = 64ll << 20;

// Device address of the static workspace on the current device (resolved
// once per device).
aol_status static_workspace(uint8_t** out);

}  // namespace aol

// Plan members use the library namespace's types unqualified.
using namespace aol;

struct aol_plan {
  int n_planes = 0;
  aol_plane_desc planes[kMaxPlanes];
  int64_t mh[kMaxPlanes], mw[kMaxPlanes];
  int elem = kU8;
  FilterHost hf, vf;
  int trx = 16, try_ = 16;
  AxisBand hb{}, vb{};
  int zpitch = 0, zrows = 0, zmb = 0;
  int xpitch = 0, xchunks = 0, rows_per_load = 0;
  LdsLayout lay{};
  size_t lds = 0;
  int grid_max = 0;  // workgroups resident on the whole device
  int slots = 0, maxk = 0, load_rounds = 1;
  int walk = 0;  // 0: row-major tiles inside a plane, 1: column-major
  // band schedule: full-width (or column-band) segments streamed down each plane
  bool use_band = false;
  int bslots = 0, bgrid = 0;
  int bseg = 0;  // requested segment (repetitions), 0: chosen per launch
  size_t blds = 0;
  FilterBands fbands;
  BandStream bstreams[kMaxPlanes];
  DeviceBuf d_bstreams;
  // Unit lists of one frame for the candidate segment lengths, longest
  // segments first, each sorted by decreasing estimated cost. Built with the
  // band schedule (plan creation, aol_plan_set_band); a launch only picks one.
  struct BandSched {
    int seg = 0;    // repetitions per segment
    int units = 0;  // units per frame
    DeviceBuf d_units;
  };
  std::vector<BandSched> bsched;
  std::string sched_json;  // text returned by aol_plan_schedule
  bool split = false;
  DeviceBuf d_hb, d_vb, d_hfrag, d_vfrag;
  // Unfused form (integer plans): one row pass per axis, each filtering
  // rows and writing them transposed; the intermediate Z^T of plane i sits
  // at byte uws_off[i] of a frame's workspace, rows uws_pitch[i] bytes apart.
  RowPassTables uh, uv;
  int64_t uws_off[kMaxPlanes] = {}, uws_pitch[kMaxPlanes] = {};
  int64_t uws_frame = 0;  // workspace bytes per frame (0: no unfused form)
  uint8_t* uws_static = nullptr;  // the static workspace on the plan's device
};
