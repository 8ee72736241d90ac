// Batched downscaling of many video streams of uneven sizes, ratios and tap
// counts in one persistent launch per step (one frame of every stream), with
// a device pointer table so the launch can be captured once in a hipGraph,
// and an autotuner for the band schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "aolmi.h"
#include "band_host.h"
#include "common.h"

using namespace aol;

namespace {

struct Schedule {
  int seg = 0;         // repetitions per segment (0: about 512 input lines)
  int budget = 150 * 1024;  // LDS budget per workgroup (picks the column band)
  std::vector<int> class_seg;  // per stream class: its own segment length (0 or absent: seg)
  // Per mille: weight of the int8-tap part's estimated cost when one launch
  // divides the device's workgroups between the two parts (the estimate
  // misjudges the two bodies' relative speed by some tens of percent).
  int part_weight = 1000;
};
constexpr int kPartWeightMin = 250, kPartWeightMax = 4000;

// Stream classes of the tuner: ratio of each axis and width class (up to
// 640, 1280, 1920 pixels, wider).
struct StreamClass {
  int hp, hq, vp, vq, wc;
  bool operator==(const StreamClass& o) const {
    return hp == o.hp && hq == o.hq && vp == o.vp && vq == o.vq && wc == o.wc;
  }
};

int width_class(int64_t w) { return w <= 640 ? 0 : w <= 1280 ? 1 : w <= 1920 ? 2 : 3; }

bool same_filter(const FilterHost& a, const FilterHost& b) {
  return a.p == b.p && a.q == b.q && a.taps == b.taps && a.c == b.c && a.s == b.s;
}

}  // namespace

struct aol_batch_plan {
  int n = 0;
  int elem = kU8;
  std::vector<aol_stream_desc> desc;  // (filter pointers are not kept)
  std::vector<FilterHost> hf, vf;
  std::vector<int> filt;              // filter group of each stream
  std::vector<int> cls;               // tuner class of each stream
  std::vector<int64_t> cls_bytes;     // input bytes of each class (the tuner's order)
  std::vector<FilterBands> bands;     // one per filter group
  // The streams whose filters fit int8 taps and those that need the split
  // operands run as two launches (each with its own kernel instance), so
  // one filter with large taps does not slow down the others.
  struct Part {
    bool split = false;
    int kmax = 0;                     // largest K-step count over the part's filter groups
    std::vector<int> ids;             // its streams
    size_t unit_capacity = 0;
    // built for the current schedule
    std::vector<BandUnit> units;
    std::vector<int64_t> cost;        // estimated cost of each unit
    int slots = 0, grid = 0;
    int resident = 0;                 // workgroups of the part's own kernel instance resident on the device
    size_t lds = 0;
    bool gather = false;
    DeviceBuf d_units, d_order, d_first;  // unit_capacity, unit_capacity, unit_capacity + 1 entries
  };
  Part parts[2];
  // Both parts in one launch (k_band_dual): each on its own share of the
  // workgroups, in proportion to its estimated cost.
  bool dual = false;
  size_t dual_lds = 0;
  Schedule sched;
  std::vector<BandStream> streams;
  DeviceBuf d_streams, d_table;
  bool pointers_set = false;
  std::string cache_path, key, sched_json;
  // Incremented by every schedule rebuild; set to kGone when the plan is
  // destroyed. Shared with the plan's graphs, which refuse to launch once it
  // differs from the value they captured.
  std::shared_ptr<uint64_t> generation = std::make_shared<uint64_t>(0);
  static constexpr uint64_t kGone = ~0ull;
  ~aol_batch_plan() { *generation = kGone; }
};

struct aol_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  DeviceBuf d_ptrs;  // a buffer-set graph's own pointer table (in, out per stream)
  std::shared_ptr<uint64_t> plan_generation;
  uint64_t captured = 0;
};

struct aol_buffer_set {
  std::shared_ptr<uint64_t> owner;  // the generation counter of the plan it was made for
  DeviceBuf d_ptrs;                 // pointer table (in, out per stream), filled at creation
};

// One part's streams, units and balanced order for a schedule.
static aol_status batch_build_part(aol_batch_plan* bp, aol_batch_plan::Part& P, const Schedule& sc,
                                   std::vector<BandStream>& streams) {
  const int n = (int)P.ids.size();
  std::vector<BandStream> ps(n);
  std::vector<const FilterBands*> fbs(n);
  for (int k = 0; k < n; ++k) fbs[k] = &bp->bands[bp->filt[P.ids[k]]];
  int lds = 0, slots = 0;
  // The part's streams share staging buffers sized for the widest, so the
  // launch may need more LDS than any one stream: narrow the column bands
  // until it fits.
  for (int budget = sc.budget;;) {
    slots = 0;
    for (int k = 0; k < n; ++k) {
      const int i = P.ids[k];
      const aol_stream_desc& d = bp->desc[i];
      int l = 0, sl = 0;
      aol_status st = build_band_stream(*fbs[k], d.height, d.width, d.in_pitch, d.out_pitch, 0, sc.seg, budget, ps[k],
                                        &l, &sl);
      if (st) return st;
      ps[k].ptr = i;
      slots = std::max(slots, sl);
    }
    std::vector<BandStream*> sp;
    for (int k = 0; k < n; ++k) sp.push_back(&ps[k]);
    lds = band_share_staging(sp.data(), fbs.data(), n);
    if (lds <= sc.budget) break;
    budget -= std::max(lds - sc.budget, 1024);
    if (budget < 8 * 1024) return fail(AOL_ERR_UNSUPPORTED, "batch streams do not fit %d bytes of LDS", sc.budget);
  }
  int wg = 0;
  hipError_t e = band_prepare(bp->elem, slots, P.split, P.kmax, (size_t)lds, &wg);
  if (e != hipSuccess) return hip_fail(e, "band kernel attributes");
  if (wg < 1) return fail(AOL_ERR_UNSUPPORTED, "batch schedule does not fit a compute unit");
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute");
  // Units in stream order (so a workgroup's units mostly share a filter),
  // assigned to workgroups by their estimated cost. Segments of the
  // schedule's length (0: about 512 input lines); a stream whose units would
  // each cost more than a workgroup's fair share gets shorter ones.
  std::vector<int> segs(n);
  for (int k = 0; k < n; ++k) {
    const int q = fbs[k]->vb.q;
    const int c = bp->cls[P.ids[k]];
    const int cs = c < (int)sc.class_seg.size() ? sc.class_seg[c] : 0;
    const int want = cs > 0 ? cs : sc.seg > 0 ? sc.seg : 16 * ((512 + 16 * q - 1) / (16 * q));
    segs[k] = std::max(16, std::min(want, band_max_seg(fbs[k]->vb)));
  }
  std::vector<BandUnit> units;
  std::vector<int64_t> cost;
  for (int round = 0; round < 8; ++round) {
    band_frame_units(ps.data(), fbs.data(), segs.data(), n, units, cost);
    int64_t total = 0;
    for (int64_t c : cost) total += c;
    const int64_t share = total / std::max<int64_t>(1, std::min<int64_t>((int64_t)wg * cus, (int64_t)units.size()));
    bool cut = false;
    for (size_t u = 0; u < units.size(); ++u) {
      const int k = units[u].stream;
      if (cost[u] > share && segs[k] > 16) {
        segs[k] = std::max(16, segs[k] / 2 / 16 * 16);
        cut = true;
        while (u + 1 < units.size() && units[u + 1].stream == k) ++u;
      }
    }
    if (!cut) break;
  }
  for (BandUnit& U : units) U.stream = P.ids[U.stream];  // index of the whole batch's descriptors
  if (units.size() > P.unit_capacity) return fail(AOL_ERR_INVALID, "unit capacity exceeded");
  P.gather = false;
  for (int k = 0; k < n; ++k) {
    streams[P.ids[k]] = ps[k];
    P.gather = P.gather || !ps[k].vec_in;
  }
  P.units = std::move(units);
  P.cost = std::move(cost);
  P.lds = (size_t)lds;
  P.slots = slots;
  P.resident = wg * cus;
  return AOL_OK;
}

// Assigns a part's units to `grid` workgroups and uploads its tables. The
// descriptor buffers keep their addresses across schedules (allocated once at
// full capacity); a graph captured before a rebuild would still run its old
// grid and kernel instance over the new tables, so aol_graph_launch refuses it
// (the plan's generation changes with every build).
static aol_status batch_place_part(aol_batch_plan::Part& P, int grid) {
  grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, (int64_t)P.units.size()));
  std::vector<int32_t> order, first;
  band_balance(P.cost, grid, order, first);
  hipError_t e;
  if ((e = hipMemcpy(P.d_units.ptr, P.units.data(), sizeof(BandUnit) * P.units.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(P.d_order.ptr, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(P.d_first.ptr, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice)) !=
          hipSuccess)
    return hip_fail(e, "hipMemcpy");
  P.grid = grid;
  return AOL_OK;
}

static aol_status batch_build(aol_batch_plan* bp, const Schedule& sc) {
  // Launches of this plan still in flight on any stream read the tables
  // rewritten below (plain copies do not wait for non-blocking streams).
  hipError_t es = hipDeviceSynchronize();
  if (es != hipSuccess) return hip_fail(es, "hipDeviceSynchronize");
  ++*bp->generation;  // first: a build that fails halfway has already rewritten tables
  std::vector<BandStream> streams(bp->n);
  int units = 0, grid = 0, lds = 0, launches = 0;
  for (aol_batch_plan::Part& P : bp->parts) {
    if (P.ids.empty()) continue;
    aol_status st = batch_build_part(bp, P, sc, streams);
    if (st) return st;
  }
  aol_batch_plan::Part &A = bp->parts[0], &B = bp->parts[1];
  const int kmax = std::max(A.kmax, B.kmax);
  bp->dual = bp->elem == kU8 && !A.ids.empty() && !B.ids.empty() && !A.gather && !B.gather &&
             band_dual_supported(A.slots, B.slots, kmax);
  if (bp->dual) {
    // one launch: the device's resident workgroups split between the parts
    // in proportion to their estimated costs
    bp->dual_lds = std::max(A.lds, B.lds);
    int wg = 0, dev = 0, cus = 0;
    hipError_t e = band_dual_prepare(A.slots, B.slots, kmax, bp->dual_lds, &wg);
    if (e != hipSuccess) return hip_fail(e, "band kernel attributes");
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return hip_fail(e, "hipDeviceGetAttribute");
    const int total = wg * cus;
    if (total < 2) return fail(AOL_ERR_UNSUPPORTED, "batch schedule does not fit a compute unit");
    double ca = 0, cb = 0;
    for (int64_t c : A.cost) ca += (double)c;
    for (int64_t c : B.cost) cb += (double)c;
    ca *= sc.part_weight / 1000.0;
    int ga = (int)(total * ca / std::max(ca + cb, 1.0) + 0.5);
    ga = std::max(1, std::min(total - 1, ga));
    aol_status st = batch_place_part(A, ga);
    if (!st) st = batch_place_part(B, total - ga);
    if (st) return st;
    units = (int)(A.units.size() + B.units.size());
    grid = A.grid + B.grid;
    lds = (int)bp->dual_lds;
    launches = 1;
  } else {
    for (aol_batch_plan::Part& P : bp->parts) {
      if (P.ids.empty()) continue;
      aol_status st = batch_place_part(P, P.resident);
      if (st) return st;
      units += (int)P.units.size();
      grid = std::max(grid, P.grid);
      lds = std::max(lds, (int)P.lds);
      ++launches;
    }
  }
  hipError_t e = hipMemcpy(bp->d_streams.ptr, streams.data(), sizeof(BandStream) * streams.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  bp->streams = std::move(streams);
  bp->sched = sc;
  char buf[240];
  snprintf(buf, sizeof buf,
           "{\"seg\": %d, \"lds_budget\": %d, \"units\": %d, \"grid\": %d, \"lds\": %d, \"launches\": %d, "
           "\"part_weight\": %d, \"class_segs\": [",
           sc.seg, sc.budget, units, grid, lds, launches, sc.part_weight);
  bp->sched_json = buf;
  for (size_t c = 0; c < sc.class_seg.size(); ++c) bp->sched_json += (c ? ", " : "") + std::to_string(sc.class_seg[c]);
  bp->sched_json += "]}";
  return AOL_OK;
}

// table: the pointer table the launch reads (NULL: the plan's)
static BandLaunch part_launch(const aol_batch_plan* bp, const aol_batch_plan::Part& P, const void* table = nullptr) {
  BandLaunch L;
  memset(&L, 0, sizeof L);
  L.streams = (const BandStream*)bp->d_streams.ptr;
  L.units = (const BandUnit*)P.d_units.ptr;
  L.units_per_frame = (int32_t)P.units.size();
  L.n_frames = 1;
  L.total_units = (int32_t)P.units.size();
  L.aligned = 1;  // checked by aol_batch_set_pointers
  L.ptr_table = (void* const*)(table ? table : bp->d_table.ptr);
  L.order = (const int32_t*)P.d_order.ptr;
  L.first = (const int32_t*)P.d_first.ptr;
  return L;
}

static aol_status batch_launch(aol_batch_plan* bp, hipStream_t stream, const void* table = nullptr) {
  if (bp->dual) {
    const aol_batch_plan::Part &A = bp->parts[0], &B = bp->parts[1];
    hipError_t e = band_dual_launch(A.slots, B.slots, std::max(A.kmax, B.kmax), part_launch(bp, A, table), A.grid,
                                    part_launch(bp, B, table), B.grid, bp->dual_lds, stream);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    return AOL_OK;
  }
  for (const aol_batch_plan::Part& P : bp->parts) {
    if (P.ids.empty()) continue;
    hipError_t e =
        band_launch(bp->elem, P.slots, P.split, P.kmax, P.gather, part_launch(bp, P, table), P.grid, P.lds, stream);
    if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  }
  return AOL_OK;
}

// Checks one buffer set (non-NULL, 16-byte aligned) and lays it out as the
// device pointer table holds it: [in_0, out_0, in_1, out_1, ...].
static aol_status batch_pointer_list(const aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                     std::vector<const void*>& ptrs) {
  if (!d_in || !d_out) return fail(AOL_ERR_INVALID, "NULL pointer array");
  ptrs.assign(2 * (size_t)plan->n, nullptr);
  for (int i = 0; i < plan->n; ++i) {
    if (!d_in[i] || !d_out[i]) return fail(AOL_ERR_INVALID, "stream %d: NULL buffer", i);
    if ((uintptr_t)d_in[i] % 16 || (uintptr_t)d_out[i] % 16)
      return fail(AOL_ERR_INVALID, "stream %d: batch buffers must be 16-byte aligned", i);
    ptrs[2 * i] = d_in[i];
    ptrs[2 * i + 1] = d_out[i];
  }
  return AOL_OK;
}

// Key of a batch for the tuning cache: device architecture, precision and
// every stream's geometry and filter.
static std::string batch_key(const aol_batch_plan* bp) {
  std::string k;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) k += prop.gcnArchName;
  k += "|" + std::to_string(bp->elem);
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the stream descriptions
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xFF);
      h *= 1099511628211ull;
    }
  };
  for (int i = 0; i < bp->n; ++i) {
    mix(bp->desc[i].height);
    mix(bp->desc[i].width);
    const FilterHost* fs[2] = {&bp->hf[i], &bp->vf[i]};
    for (const FilterHost* f : fs) {
      mix(f->p);
      mix(f->q);
      mix(f->taps);
      for (int c : f->c) mix(c);
      for (int s : f->s) mix(s);
    }
  }
  char buf[32];
  snprintf(buf, sizeof buf, "|%016llx", (unsigned long long)h);
  return k + buf;
}

// Tiny line-oriented cache: "key seg budget n_classes class_seg... part_weight"
// per line (the last line of a key wins; a line without the weight: 1000).
static bool cache_lookup(const std::string& path, const std::string& key, Schedule* sc) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[400];
    int seg = 0, budget = 0, used = 0;
    if (sscanf(line, "%399s %d %d%n", k, &seg, &budget, &used) == 3 && key == k) {
      sc->seg = seg;
      sc->budget = budget;
      sc->class_seg.clear();
      sc->part_weight = 1000;
      int n = 0, m = 0;
      const char* rest = line + used;
      if (sscanf(rest, "%d%n", &n, &m) == 1 && n >= 0 && n <= 4096) {
        rest += m;
        int c = 0;
        for (; c < n; ++c) {
          int v = 0;
          if (sscanf(rest, "%d%n", &v, &m) != 1) break;
          rest += m;
          sc->class_seg.push_back(v);
        }
        int wgt = 0;
        if (c == n && sscanf(rest, "%d", &wgt) == 1 && wgt >= kPartWeightMin && wgt <= kPartWeightMax)
          sc->part_weight = wgt;
      }
      found = true;
    }
  }
  fclose(f);
  return found;
}

static void cache_store(const std::string& path, const std::string& key, const Schedule& sc) {
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d", key.c_str(), sc.seg, sc.budget, (int)sc.class_seg.size());
  for (int v : sc.class_seg) fprintf(f, " %d", v);
  fprintf(f, " %d\n", sc.part_weight);
  fclose(f);
}

extern "C" {

aol_status aol_batch_plan_create(int32_t n_streams, const aol_stream_desc* streams, aol_precision prec,
                                 const char* tune_cache, aol_batch_plan** out) {
  if (!out) return fail(AOL_ERR_INVALID, "NULL plan output");
  *out = nullptr;
  if (n_streams < 1 || !streams) return fail(AOL_ERR_INVALID, "need at least one stream");
  if (n_streams > 4096) return fail(AOL_ERR_UNSUPPORTED, "at most 4096 streams");
  if (prec != AOL_PREC_U8 && prec != AOL_PREC_BF16 && prec != AOL_PREC_FP16)
    return fail(AOL_ERR_INVALID, "unknown precision %d", (int)prec);
  aol_batch_plan* bp = new (std::nothrow) aol_batch_plan();
  if (!bp) return fail(AOL_ERR_NOMEM, "plan allocation");
  bp->n = n_streams;
  bp->elem = prec == AOL_PREC_U8 ? kU8 : prec == AOL_PREC_BF16 ? kBF16 : kFP16;
  bp->desc.assign(streams, streams + n_streams);
  bp->hf.resize(n_streams);
  bp->vf.resize(n_streams);
  bp->filt.resize(n_streams);
  aol_status st = AOL_OK;
  for (int i = 0; i < n_streams && !st; ++i) {
    aol_stream_desc& d = bp->desc[i];
    if (d.height < 1 || d.width < 1 || d.height > (1 << 30) || d.width > (1 << 30)) {
      st = fail(AOL_ERR_INVALID, "stream %d: size %lldx%lld", i, (long long)d.height, (long long)d.width);
      break;
    }
    if ((st = check_filter(&streams[i].hf, "hf", bp->hf[i]))) break;
    if ((st = check_filter(&streams[i].vf, "vf", bp->vf[i]))) break;
    const int64_t mw = (int64_t)bp->hf[i].p * ((d.width + bp->hf[i].q - 1) / bp->hf[i].q);
    if (d.in_pitch == 0) d.in_pitch = d.width;
    if (d.out_pitch == 0) d.out_pitch = mw;
    if (d.in_pitch < d.width || d.out_pitch < mw) {
      st = fail(AOL_ERR_INVALID, "stream %d: pitch smaller than the row", i);
      break;
    }
    d.hf.coeff = nullptr;
    d.hf.phase_start = nullptr;
    d.vf.coeff = nullptr;
    d.vf.phase_start = nullptr;
  }
  if (st) {
    delete bp;
    return st;
  }
  // filter groups; the groups that need the split integer taps go to the
  // second launch
  std::vector<int> rep;
  for (int i = 0; i < n_streams; ++i) {
    int gidx = -1;
    for (size_t g = 0; g < rep.size(); ++g)
      if (same_filter(bp->hf[rep[g]], bp->hf[i]) && same_filter(bp->vf[rep[g]], bp->vf[i])) gidx = (int)g;
    if (gidx < 0) {
      gidx = (int)rep.size();
      rep.push_back(i);
    }
    bp->filt[i] = gidx;
  }
  bp->bands.clear();
  bp->bands.resize(rep.size());
  for (size_t g = 0; g < rep.size(); ++g) {
    st = build_filter_bands(bp->hf[rep[g]], bp->vf[rep[g]], bp->elem, false, bp->bands[g]);
    if (st) {
      delete bp;
      return st;
    }
  }
  for (int i = 0; i < n_streams; ++i) {
    const FilterBands& fb = bp->bands[bp->filt[i]];
    aol_batch_plan::Part& P = bp->parts[fb.split ? 1 : 0];
    P.split = fb.split;
    P.kmax = std::max(P.kmax, fb.kmax);
    P.ids.push_back(i);
  }
  // tuner classes (ratios, width class), ordered by their input bytes
  {
    std::vector<StreamClass> cl;
    bp->cls.resize(n_streams);
    for (int i = 0; i < n_streams; ++i) {
      const StreamClass c{bp->hf[i].p, bp->hf[i].q, bp->vf[i].p, bp->vf[i].q, width_class(bp->desc[i].width)};
      size_t j = 0;
      while (j < cl.size() && !(cl[j] == c)) ++j;
      if (j == cl.size()) {
        cl.push_back(c);
        bp->cls_bytes.push_back(0);
      }
      bp->cls[i] = (int)j;
      bp->cls_bytes[j] += bp->desc[i].height * bp->desc[i].width;
    }
  }
  bp->key = batch_key(bp);
  Schedule sc;
  if (tune_cache) {
    bp->cache_path = tune_cache;
    cache_lookup(bp->cache_path, bp->key, &sc);
  }
  // capacity: the most units any schedule can make (bands and segments of 16 repetitions)
  st = AOL_OK;
  for (aol_batch_plan::Part& P : bp->parts) {
    for (int i : P.ids) {
      const int64_t rx = (bp->desc[i].width + bp->hf[i].q - 1) / bp->hf[i].q;
      const int64_t ry = (bp->desc[i].height + bp->vf[i].q - 1) / bp->vf[i].q;
      P.unit_capacity += (size_t)(((rx + 15) / 16) * ((ry + 15) / 16));
    }
    if (P.unit_capacity > (size_t)INT_MAX / 2) {
      delete bp;
      return fail(AOL_ERR_UNSUPPORTED, "too many units");
    }
    if (P.ids.empty()) continue;
    if (!st) st = P.d_units.alloc(sizeof(BandUnit) * P.unit_capacity);
    if (!st) st = P.d_order.alloc(sizeof(int32_t) * P.unit_capacity);
    if (!st) st = P.d_first.alloc(sizeof(int32_t) * (P.unit_capacity + 1));
  }
  if (!st) st = bp->d_streams.alloc(sizeof(BandStream) * (size_t)n_streams);
  if (!st) st = batch_build(bp, sc);
  if (!st) st = bp->d_table.alloc(sizeof(void*) * 2 * (size_t)n_streams);
  if (st) {
    delete bp;
    return st;
  }
  *out = bp;
  return ok();
}

aol_status aol_batch_plan_destroy(aol_batch_plan* plan) {
  delete plan;
  return ok();
}

aol_status aol_batch_set_pointers(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                  hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  std::vector<const void*> ptrs;
  if (aol_status st = batch_pointer_list(plan, d_in, d_out, ptrs)) return st;
  hipError_t e = set_pointers_launch((void**)plan->d_table.ptr, ptrs.data(), 2 * plan->n, stream);
  if (e != hipSuccess) return hip_fail(e, "pointer table update");
  plan->pointers_set = true;
  return ok();
}

aol_status aol_batch_run(aol_batch_plan* plan, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (!plan->pointers_set) return fail(AOL_ERR_INVALID, "aol_batch_set_pointers was never called");
  aol_status st = batch_launch(plan, stream);
  return st ? st : ok();
}

aol_status aol_batch_buffers_create(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                    aol_buffer_set** out) {
  if (!plan || !out) return fail(AOL_ERR_INVALID, "NULL argument");
  *out = nullptr;
  std::vector<const void*> ptrs;
  if (aol_status st = batch_pointer_list(plan, d_in, d_out, ptrs)) return st;
  aol_buffer_set* b = new (std::nothrow) aol_buffer_set();
  if (!b) return fail(AOL_ERR_NOMEM, "buffer set allocation");
  b->owner = plan->generation;
  if (aol_status st = b->d_ptrs.upload(ptrs.data(), ptrs.size() * sizeof(void*))) {
    delete b;
    return st;
  }
  *out = b;
  return ok();
}

aol_status aol_batch_run_buffers(aol_batch_plan* plan, const aol_buffer_set* set, hipStream_t stream) {
  if (!plan || !set) return fail(AOL_ERR_INVALID, "NULL argument");
  if (set->owner != plan->generation) return fail(AOL_ERR_INVALID, "the buffer set was made for another plan");
  aol_status st = batch_launch(plan, stream, set->d_ptrs.ptr);
  return st ? st : ok();
}

aol_status aol_batch_buffers_destroy(aol_buffer_set* set) {
  delete set;
  return ok();
}

}  // extern "C"

// Captures one batch launch into a graph; with `ptrs` the graph gets its own
// pointer table holding them (filled now), which its launch reads.
static aol_status batch_graph_capture(aol_batch_plan* plan, const std::vector<const void*>* ptrs, hipStream_t stream,
                                      aol_graph** out) {
  if (!stream) return fail(AOL_ERR_INVALID, "graph capture needs a non-default stream");
  aol_graph* g = new (std::nothrow) aol_graph();
  if (!g) return fail(AOL_ERR_NOMEM, "graph allocation");
  if (ptrs) {
    if (aol_status st = g->d_ptrs.upload(ptrs->data(), ptrs->size() * sizeof(void*))) {
      delete g;
      return st;
    }
  }
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  aol_status st = batch_launch(plan, stream, ptrs ? g->d_ptrs.ptr : nullptr);
  e = hipStreamEndCapture(stream, &g->graph);
  if (st || e != hipSuccess) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st ? st : hip_fail(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(e, "hipGraphInstantiate");
  }
  g->plan_generation = plan->generation;
  g->captured = *plan->generation;
  *out = g;
  return AOL_OK;
}

extern "C" {

aol_status aol_batch_graph_create(aol_batch_plan* plan, hipStream_t stream, aol_graph** out) {
  if (!plan || !out) return fail(AOL_ERR_INVALID, "NULL argument");
  *out = nullptr;
  aol_status st = batch_graph_capture(plan, nullptr, stream, out);
  return st ? st : ok();
}

aol_status aol_batch_graph_create_pointers(aol_batch_plan* plan, const void* const* d_in, void* const* d_out,
                                           hipStream_t stream, aol_graph** out) {
  if (!plan || !out) return fail(AOL_ERR_INVALID, "NULL argument");
  *out = nullptr;
  std::vector<const void*> ptrs;
  aol_status st = batch_pointer_list(plan, d_in, d_out, ptrs);
  if (!st) st = batch_graph_capture(plan, &ptrs, stream, out);
  return st ? st : ok();
}

aol_status aol_graph_launch(aol_graph* graph, hipStream_t stream) {
  if (!graph || !graph->exec) return fail(AOL_ERR_INVALID, "NULL graph");
  if (*graph->plan_generation != graph->captured)
    return fail(AOL_ERR_INVALID, *graph->plan_generation == aol_batch_plan::kGone
                                     ? "the graph's batch plan was destroyed"
                                     : "the batch plan's schedule changed (aol_autotune) since this graph was captured");
  hipError_t e = hipGraphLaunch(graph->exec, stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

aol_status aol_graph_destroy(aol_graph* graph) {
  if (graph) {
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
  }
  return ok();
}

// Time of one launch of a schedule: after one warm-up, three groups of three
// launches back to back, each group between two events; the fastest group's
// mean (robust to a group slowed by something else on the device). A negative
// time when the schedule does not fit.
static aol_status time_schedule(aol_batch_plan* plan, const Schedule& sc, hipStream_t stream, hipEvent_t e0,
                                hipEvent_t e1, float* ms) {
  *ms = -1.f;
  if (batch_build(plan, sc) != AOL_OK) return AOL_OK;  // candidate does not fit
  aol_status st = batch_launch(plan, stream);           // warm-up
  if (st) return st;
  float best = -1.f;
  for (int g = 0; g < 3; ++g) {
    hipError_t e;
    if ((e = hipEventRecord(e0, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int r = 0; r < 3 && !st; ++r) st = batch_launch(plan, stream);
    if (st) return st;
    if ((e = hipEventRecord(e1, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    if (best < 0.f || t < best) best = t;
  }
  *ms = best / 3.f;
  return AOL_OK;
}

aol_status aol_autotune(aol_batch_plan* plan, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (!plan->pointers_set) return fail(AOL_ERR_INVALID, "aol_autotune needs aol_batch_set_pointers first");
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  Schedule best = plan->sched;
  float best_ms = 1e30f;
  aol_status st = AOL_OK;
  auto trial = [&](const Schedule& sc) {
    float ms = 0.f;
    st = time_schedule(plan, sc, stream, e0, e1, &ms);
    if (!st && ms >= 0.f && ms < best_ms) {
      best_ms = ms;
      best = sc;
    }
    return st == AOL_OK;
  };
  // the weight of the int8-tap part when both parts share one launch
  auto weights = [&](std::initializer_list<int> deltas) {
    if (best_ms >= 1e30f || batch_build(plan, best) != AOL_OK || !plan->dual) return true;
    const Schedule base = best;
    for (int d : deltas) {
      Schedule sc = base;
      sc.part_weight = base.part_weight + d;
      if (sc.part_weight < kPartWeightMin || sc.part_weight > kPartWeightMax) continue;
      if (!trial(sc)) return false;
    }
    return true;
  };
  // 1. one segment length and LDS budget (column band) for every stream
  const int segs[] = {16, 32, 64, 128};
  const int budgets[] = {150 * 1024, 76 * 1024};
  bool go = true;
  for (int budget : budgets)
    for (int seg : segs) {
      Schedule sc;
      sc.seg = seg;
      sc.budget = budget;
      if (go) go = trial(sc);
    }
  // 2. the parts' weight, coarse
  if (go) go = weights({-500, -400, -300, -200, -100, 100, 250, 500});
  // 3. each stream class's own segment length, classes with the most input
  // first, the others held at their best so far (one pass)
  if (go && best_ms < 1e30f) {
    std::vector<int> order(plan->cls_bytes.size());
    for (size_t c = 0; c < order.size(); ++c) order[c] = (int)c;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return plan->cls_bytes[a] > plan->cls_bytes[b]; });
    best.class_seg.assign(order.size(), 0);
    const int class_segs[] = {16, 32, 48, 64, 96, 128};
    for (int c : order) {
      const Schedule base = best;
      for (int seg : class_segs) {
        Schedule sc = base;
        sc.class_seg[c] = seg;
        if (go) go = trial(sc);
      }
    }
  }
  // 4. the parts' weight again, fine, around the best
  if (go) go = weights({-100, -50, 50, 100});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if ((st = batch_build(plan, best))) return st;
  if (!plan->cache_path.empty()) cache_store(plan->cache_path, plan->key, best);
  return ok();
}

aol_status aol_batch_set_schedule(aol_batch_plan* plan, int32_t seg_reps, int32_t lds_budget) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (seg_reps < 0 || seg_reps % 16) return fail(AOL_ERR_INVALID, "seg_reps must be a multiple of 16 (or 0)");
  if (lds_budget < 16 * 1024 || lds_budget > 160 * 1024)
    return fail(AOL_ERR_INVALID, "lds_budget must be within 16 KiB .. 160 KiB");
  Schedule sc;
  sc.seg = seg_reps;
  sc.budget = lds_budget;
  aol_status st = batch_build(plan, sc);
  if (st) {
    const std::string msg = last_error();
    const Schedule old = plan->sched;
    if (batch_build(plan, old) != AOL_OK) return fail(AOL_ERR_HIP, "restoring the previous schedule failed");
    return fail(st, "%s", msg.c_str());
  }
  return ok();
}

aol_status aol_batch_set_part_weight(aol_batch_plan* plan, int32_t permille) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (permille < kPartWeightMin || permille > kPartWeightMax)
    return fail(AOL_ERR_INVALID, "part weight must be within %d .. %d per mille", kPartWeightMin, kPartWeightMax);
  const Schedule old = plan->sched;
  Schedule sc = old;
  sc.part_weight = permille;
  aol_status st = batch_build(plan, sc);
  if (st) {
    const std::string msg = last_error();
    if (batch_build(plan, old) != AOL_OK) return fail(AOL_ERR_HIP, "restoring the previous schedule failed");
    return fail(st, "%s", msg.c_str());
  }
  return ok();
}

const char* aol_batch_schedule(aol_batch_plan* plan) {
  return plan ? plan->sched_json.c_str() : "";
}

}  // extern "C"
