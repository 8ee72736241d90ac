// Host side of the downscaler: validation, per-axis band tables, plans and
// the C ABI entry points declared in include/aolmi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "aol_internal.h"
#include "aolmi.h"
#include "band_host.h"
#include "common.h"
#include "plan.h"

namespace aol {

hipError_t fused_prepare(int elem, bool split, int slots, int maxk, size_t lds_bytes, int* wg_per_cu);
hipError_t fused_launch(int elem, bool split, int slots, int maxk, const FusedArgs& a, int grid, size_t lds_bytes,
                        hipStream_t stream);

static thread_local std::string g_err;

aol_status fail(aol_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

aol_status ok() {
  g_err.clear();
  return AOL_OK;
}

aol_status hip_fail(hipError_t e, const char* what) {
  return fail(AOL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

static int64_t pmod64(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

void default_starts(int p, int q, int taps, int32_t* out) {
  // The output pixel of phase phi is centred at input coordinate
  // ((2phi+1)q - p) / (2p) (pixel centres at integer positions); the window
  // of `taps` pixels starts floor((taps-1)/2) before the pixel under it.
  for (int phi = 0; phi < p; ++phi)
    out[phi] = (int32_t)(floor_div((int64_t)(2 * phi + 1) * q - p, 2LL * p) - (taps - 1) / 2);
}

aol_status check_filter(const aol_polyphase* f, const char* name, FilterHost& out) {
  if (!f) return fail(AOL_ERR_INVALID, "%s: NULL filter", name);
  if (f->p < 1 || f->q < 1 || f->taps < 1) return fail(AOL_ERR_INVALID, "%s: p, q and taps must be >= 1", name);
  if (!f->coeff) return fail(AOL_ERR_INVALID, "%s: NULL coefficients", name);
  if (f->p > AOL_MAX_P) return fail(AOL_ERR_UNSUPPORTED, "%s: p=%d exceeds %d", name, f->p, AOL_MAX_P);
  if (f->q > AOL_MAX_Q) return fail(AOL_ERR_UNSUPPORTED, "%s: q=%d exceeds %d", name, f->q, AOL_MAX_Q);
  if (f->taps > AOL_MAX_TAPS) return fail(AOL_ERR_UNSUPPORTED, "%s: taps=%d exceeds %d", name, f->taps, AOL_MAX_TAPS);
  out.p = f->p;
  out.q = f->q;
  out.taps = f->taps;
  out.c.assign(f->coeff, f->coeff + (size_t)f->p * f->taps);
  out.s.resize(f->p);
  if (f->phase_start) {
    for (int i = 0; i < f->p; ++i) {
      if (f->phase_start[i] < -4096 || f->phase_start[i] > 4096)
        return fail(AOL_ERR_UNSUPPORTED, "%s: phase_start[%d]=%d outside [-4096, 4096]", name, i, f->phase_start[i]);
      out.s[i] = f->phase_start[i];
    }
  } else {
    default_starts(f->p, f->q, f->taps, out.s.data());
  }
  return AOL_OK;
}

static uint16_t f32_to_bf16_exact(float x, bool* exact) {
  uint32_t u;
  memcpy(&u, &x, 4);
  *exact = (u & 0xFFFFu) == 0;
  return (uint16_t)(u >> 16);
}

static uint16_t f32_to_f16_exact(float x, bool* exact) {
  // Exact conversion for the values used here (c/256 with |c| <= 2047):
  // normal fp16 covers 2^-14 .. 65504 with 11 significant bits.
  _Float16 h = (_Float16)x;
  *exact = ((float)h == x);
  uint16_t r;
  memcpy(&r, &h, 2);
  return r;
}

aol_status build_band(const FilterHost& f, int tr, int elem, bool h_axis, bool force_split, AxisBand& band,
                      std::vector<uint8_t>& frags, const char* name) {
  memset(&band, 0, sizeof band);
  const int E = elem == kU8 ? 16 : 8;
  const int p = f.p, q = f.q, T = f.taps;
  int s_min = INT_MAX, s_end = INT_MIN;
  for (int phi = 0; phi < p; ++phi) {
    s_min = std::min(s_min, f.s[phi]);
    s_end = std::max(s_end, f.s[phi] + T);
  }
  band.p = p;
  band.q = q;
  band.taps = T;
  band.tr = tr;
  band.n_out = p * tr;
  band.nblk = (band.n_out + 15) / 16;
  band.span = s_end - s_min;
  band.s_min = s_min;
  band.delta = h_axis ? (int)pmod64(s_min, E) : 0;
  band.chunk_elems = E;
  if (band.nblk > kMaxNB) return fail(AOL_ERR_UNSUPPORTED, "%s: %d outputs per tile exceed %d", name, band.n_out, kMaxNB * 16);
  if (h_axis && (q * tr) % E != 0) return fail(AOL_ERR_INVALID, "%s: q*tile must be a multiple of %d", name, E);

  bool split = false;
  if (elem == kU8) {
    for (int v : f.c) {
      if (v < -AOL_MAX_COEFF || v > AOL_MAX_COEFF)
        return fail(AOL_ERR_UNSUPPORTED, "%s: coefficient %d outside +-%d", name, v, AOL_MAX_COEFF);
      if (v < -128 || v > 127) split = true;
    }
  } else {
    for (int v : f.c) {
      bool exact = false;
      if (elem == kBF16) f32_to_bf16_exact((float)v / 256.0f, &exact);
      else f32_to_f16_exact((float)v / 256.0f, &exact);
      if (v < -AOL_MAX_COEFF || v > AOL_MAX_COEFF || !exact)
        return fail(AOL_ERR_UNSUPPORTED, "%s: coefficient %d/256 is not exact in the %s format", name, v,
                    elem == kBF16 ? "bf16" : "fp16");
    }
  }
  split = split || (elem == kU8 && force_split);
  band.split = split ? 1 : 0;

  // Per output block: the window of tile-local element positions (position 0
  // is the start of the tile's first chunk) its outputs read.
  int nfrag = 0;
  int chunk_hi = 0;
  frags.clear();
  for (int b = 0; b < band.nblk; ++b) {
    int lo = INT_MAX, hi = INT_MIN;
    for (int o = 16 * b; o < std::min(16 * b + 16, band.n_out); ++o) {
      const int r = o / p, phi = o % p;
      const int st = band.delta + q * r + f.s[phi] - s_min;
      lo = std::min(lo, st);
      hi = std::max(hi, st + T);
    }
    band.wend[b] = hi;
    const int c0 = lo / E;
    const int c1 = (hi + E - 1) / E;
    const int nk = (c1 - c0 + 3) / 4;
    if (nk > kMaxK)
      return fail(AOL_ERR_UNSUPPORTED, "%s: a block of 16 outputs spans %d input elements (at most %d)", name,
                  hi - lo, kMaxK * 4 * E - (E - 1));
    band.chunk0[b] = c0;
    band.nk[b] = nk;
    band.frag[b] = nfrag;
    chunk_hi = std::max(chunk_hi, c0 + 4 * nk);
    const size_t blk_begin = frags.size();
    for (int kb = 0; kb < nk; ++kb) {
      const int parts = split ? 2 : 1;
      const size_t base = frags.size();
      frags.resize(base + (size_t)parts * kLanes * 16, 0);
      for (int lane = 0; lane < kLanes; ++lane) {
        const int g = lane >> 4, nn = lane & 15;
        const int o = 16 * b + nn;
        for (int e = 0; e < E; ++e) {
          const int k = (c0 + 4 * kb + g) * E + e;
          int c = 0;
          if (o < band.n_out) {
            const int r = o / p, phi = o % p;
            const int t = k - (band.delta + q * r + f.s[phi] - s_min);
            if (t >= 0 && t < T) c = f.c[(size_t)phi * T + t];
          }
          if (elem == kU8) {
            const int lo7 = (int)pmod64(c + 64, 128) - 64;  // c = lo7 + 128*hi
            const int hi7 = (c - lo7) / 128;
            frags[base + (size_t)lane * 16 + e] = (uint8_t)(int8_t)(split ? lo7 : c);
            if (split) frags[base + (size_t)kLanes * 16 + (size_t)lane * 16 + e] = (uint8_t)(int8_t)hi7;
          } else {
            bool exact;
            const uint16_t bits = elem == kBF16 ? f32_to_bf16_exact((float)c / 256.0f, &exact)
                                                : f32_to_f16_exact((float)c / 256.0f, &exact);
            memcpy(&frags[base + (size_t)lane * 16 + 2 * e], &bits, 2);
          }
        }
      }
      nfrag += 1;
    }
    // Blocks repeat with the band's period (p outputs per q inputs): reuse an
    // identical earlier fragment run instead of storing it again.
    {
      const size_t len = frags.size() - blk_begin;
      const size_t fbytes = (size_t)(split ? 2 : 1) * kLanes * 16;
      for (int pb = 0; pb < b; ++pb) {
        if (band.nk[pb] != nk) continue;
        const size_t off = (size_t)band.frag[pb] * fbytes;
        if (memcmp(&frags[off], &frags[blk_begin], len) == 0) {
          frags.resize(blk_begin);
          nfrag -= nk;
          band.frag[b] = band.frag[pb];
          break;
        }
      }
    }
    for (int nn = 0; nn < 16; ++nn) {
      const int o = 16 * b + nn;
      int64_t S = 0;
      if (o < band.n_out) {
        const int phi = o % p;
        for (int t = 0; t < T; ++t) S += f.c[(size_t)phi * T + t];
      }
      band.bias[b * 16 + nn] = (int32_t)(128 * S + 128);
    }
  }
  band.nchunks = chunk_hi;
  // one all-zero fragment (pair) after the others: the operand of the K-steps
  // a block does not need when every block runs the same number of them
  band.zfrag = nfrag;
  frags.resize(frags.size() + (size_t)(split ? 2 : 1) * kLanes * 16, 0);
  nfrag += 1;
  band.nfrag = nfrag * (split ? 2 : 1);
  band.kmax = 0;
  for (int b = 0; b < band.nblk; ++b) band.kmax = std::max(band.kmax, band.nk[b]);
  band.ubias = 1;
  for (int i = 0; i < band.nblk * 16; ++i) band.ubias = band.ubias && band.bias[i] == band.bias[0];
  return AOL_OK;
}

}  // namespace aol

using namespace aol;


static int gcd_int(int a, int b) {
  while (b) {
    const int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Repetitions per tile along one axis: about 128 input elements, a whole
// number of 16-byte chunks along lines, at most kMaxNB*16 outputs.
static int tile_align(const FilterHost& f, int elem, bool h_axis) {
  const int E = elem == kU8 ? 16 : 8;
  return h_axis ? E / gcd_int(f.q, E) : 1;
}

static int default_tile(const FilterHost& f, int elem, bool h_axis, int target = 128) {
  const int al = tile_align(f, elem, h_axis);
  int tr = (target + f.q - 1) / f.q;
  tr = (tr + al - 1) / al * al;
  const int cap = std::max(al, (kMaxNB * 16 / f.p) / al * al);
  return std::max(1, std::min(tr, cap));
}

static aol_status plan_build_tables(aol_plan* pl, int trx, int try_) {
  AxisBand hb, vb;
  std::vector<uint8_t> hfr, vfr;
  aol_status st = build_band(pl->hf, trx, pl->elem, true, false, hb, hfr, "hf");
  if (st) return st;
  st = build_band(pl->vf, try_, pl->elem, false, hb.split != 0, vb, vfr, "vf");
  if (st) return st;
  if (vb.split && !hb.split) {  // one kernel instance carries both axes: same operand layout
    st = build_band(pl->hf, trx, pl->elem, true, true, hb, hfr, "hf");
    if (st) return st;
  }
  const int E = pl->elem == kU8 ? 16 : 8;
  const int es = pl->elem == kU8 ? 1 : 2;
  // Intermediate lines the vertical pass may read (all K-steps of a full tile).
  const int zlines = ((vb.nchunks * E) + 15) / 16 * 16;
  int zpitch = zlines;
  if (((zpitch * es) / 16) % 2 == 0) zpitch += 16 / es;  // odd multiple of 16 bytes between LDS rows
  const int zrows = hb.nblk * 16;
  // Input tile: the lines of a full tile by the chunks any horizontal K-step reads.
  const int xchunks = hb.nchunks;
  if (xchunks > 64) return fail(AOL_ERR_UNSUPPORTED, "tile rows of %d chunks exceed 64", xchunks);
  int xpitch = xchunks * 16;
  if ((xpitch / 16) % 2 == 0) xpitch += 16;
  const int xrows = vb.q * (try_ - 1) + vb.span;
  const int rpl = 64 / xchunks;
  const int slots = (xrows + rpl * kWaves - 1) / (rpl * kWaves);  // loads per lane for one input tile
  int maxk = 1;
  for (int b = 0; b < hb.nblk; ++b) maxk = std::max(maxk, hb.nk[b]);
  for (int b = 0; b < vb.nblk; ++b) maxk = std::max(maxk, vb.nk[b]);
  const bool split = hb.split || vb.split;
  LdsLayout lay;
  lay.frag_h = 0;
  lay.frag_v = lay.frag_h + hb.nfrag * kLanes * 16;
  lay.bias_h = lay.frag_v + vb.nfrag * kLanes * 16;
  lay.bias_v = lay.bias_h + hb.nblk * 16 * 4;
  lay.x = (lay.bias_v + vb.nblk * 16 * 4 + 15) / 16 * 16;
  lay.z = lay.x + xrows * xpitch;
  lay.total = lay.z + zrows * zpitch * es * (pl->elem == kU8 ? 1 : 2);
  const size_t lds = (size_t)lay.total;
  if (lds > 160 * 1024) return fail(AOL_ERR_UNSUPPORTED, "tile %dx%d needs %zu bytes of LDS", trx, try_, lds);
  int wg_per_cu = 0;
  hipError_t e = fused_prepare(pl->elem, split, slots, maxk, lds, &wg_per_cu);
  if (e != hipSuccess) return hip_fail(e, "fused kernel attributes");
  if (wg_per_cu < 1) return fail(AOL_ERR_UNSUPPORTED, "tile %dx%d does not fit a compute unit", trx, try_);
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute");
  DeviceBuf dhb, dvb, dhf, dvf;
  if ((st = dhb.upload(&hb, sizeof hb))) return st;
  if ((st = dvb.upload(&vb, sizeof vb))) return st;
  if ((st = dhf.upload(hfr.data(), hfr.size()))) return st;
  if ((st = dvf.upload(vfr.data(), vfr.size()))) return st;
  pl->hb = hb;
  pl->vb = vb;
  pl->trx = trx;
  pl->try_ = try_;
  pl->zpitch = zpitch;
  pl->zrows = zrows;
  pl->zmb = zlines / 16;
  pl->xpitch = xpitch;
  pl->xchunks = xchunks;
  pl->rows_per_load = rpl;
  pl->lay = lay;
  pl->lds = lds;
  pl->grid_max = wg_per_cu * cus;
  pl->slots = slots;
  pl->load_rounds = slots <= 6 ? 1 : (slots + kMaxSlots - 1) / kMaxSlots;
  pl->maxk = maxk;
  pl->split = split;
  pl->d_hb = std::move(dhb);
  pl->d_vb = std::move(dvb);
  pl->d_hfrag = std::move(dhf);
  pl->d_vfrag = std::move(dvf);
  return AOL_OK;
}

namespace aol {

aol_status build_rowpass_tables(const FilterHost& f, RowPassTables& out, const char* name) {
  std::vector<uint8_t> fr;
  AxisBand b;
  aol_status st = build_band(f, 16, kU8, true, false, b, fr, name);
  if (st) return st;
  out.band = b;
  out.x0 = b.s_min - b.delta;
  if ((st = out.d_band.upload(&b, sizeof b))) return st;
  return out.d_frag.upload(fr.data(), fr.size());
}

}  // namespace aol

// The unfused form of an integer plan: both axes' row-pass tables and the
// layout of one frame's transposed intermediates (rows padded to whole
// 128-byte lines, planes 256-byte aligned).
static aol_status plan_build_unfused(aol_plan* pl) {
  pl->uws_frame = 0;
  aol_status st = build_rowpass_tables(pl->hf, pl->uh, "hf");
  if (!st) st = build_rowpass_tables(pl->vf, pl->uv, "vf");
  if (st) return st == AOL_ERR_UNSUPPORTED ? AOL_OK : st;  // filters beyond the row pass: no unfused form
  int64_t off = 0;
  for (int i = 0; i < pl->n_planes; ++i) {
    pl->uws_off[i] = off;
    pl->uws_pitch[i] = (pl->planes[i].height + 127) / 128 * 128;
    off += (pl->mw[i] * pl->uws_pitch[i] + 255) / 256 * 256;
  }
  pl->uws_frame = off;
  return static_workspace(&pl->uws_static);
}

// The band schedule (default): one workgroup per column band of a plane,
// streaming segments down it. Budget: one workgroup of LDS per compute unit.
static constexpr int kBandLdsBudget = 150 * 1024;

static aol_status plan_build_band(aol_plan* pl, int xreps, int seg) {
  pl->use_band = false;
  FilterBands fb;
  aol_status st = build_filter_bands(pl->hf, pl->vf, pl->elem, false, fb);
  if (st) return st == AOL_ERR_UNSUPPORTED ? AOL_OK : st;
  int lds = 0, slots = 0;
  for (int i = 0; i < pl->n_planes; ++i) {
    int l = 0, sl = 0;
    st = build_band_stream(fb, pl->planes[i].height, pl->planes[i].width, pl->planes[i].in_pitch,
                           pl->planes[i].out_pitch, xreps, seg, kBandLdsBudget, pl->bstreams[i], &l, &sl);
    if (st) return st == AOL_ERR_UNSUPPORTED ? AOL_OK : st;
    pl->bstreams[i].ptr = i;
    lds = std::max(lds, l);
    slots = std::max(slots, sl);
  }
  {
    std::vector<BandStream*> sp;
    std::vector<const FilterBands*> fp;
    for (int i = 0; i < pl->n_planes; ++i) {
      sp.push_back(&pl->bstreams[i]);
      fp.push_back(&fb);
    }
    lds = band_share_staging(sp.data(), fp.data(), pl->n_planes);
    if (lds > kBandLdsBudget) return AOL_OK;
  }
  int wg = 0;
  hipError_t e = band_prepare(pl->elem, slots, fb.split, fb.kmax, (size_t)lds, &wg);
  if (e != hipSuccess) return hip_fail(e, "band kernel attributes");
  if (wg < 1) return AOL_OK;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute");
  DeviceBuf ds;
  if ((st = ds.upload(pl->bstreams, sizeof(BandStream) * pl->n_planes))) return st;
  // Segment lengths: the requested one, else about 512, 256, 128 and 64 input
  // lines. Each list holds the units of one frame, most expensive first: a
  // launch over n frames hands its n * units items to the workgroups in
  // rounds (see k_band), so the list never depends on the frame count.
  std::vector<aol_plan::BandSched> scheds;
  {
    const FilterBands* fbs[kMaxPlanes];
    for (int i = 0; i < pl->n_planes; ++i) fbs[i] = &fb;
    const AxisBand& vb = fb.vb;
    for (int lines = 512; lines >= 64; lines /= 2) {
      int sg = seg > 0 ? seg : 16 * ((lines + 16 * vb.q - 1) / (16 * vb.q));
      sg = std::max(16, std::min(sg, band_max_seg(vb)));
      if (!scheds.empty() && scheds.back().seg == sg) continue;
      int segs[kMaxPlanes];
      for (int i = 0; i < pl->n_planes; ++i) segs[i] = sg;
      std::vector<BandUnit> units;
      std::vector<int64_t> cost;
      band_frame_units(pl->bstreams, fbs, segs, pl->n_planes, units, cost);
      std::vector<int> idx(units.size());
      for (size_t u = 0; u < idx.size(); ++u) idx[u] = (int)u;
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
      std::vector<BandUnit> sorted;
      for (int u : idx) sorted.push_back(units[u]);
      aol_plan::BandSched sc;
      sc.seg = sg;
      sc.units = (int)sorted.size();
      if ((st = sc.d_units.upload(sorted.data(), sizeof(BandUnit) * sorted.size()))) return st;
      scheds.push_back(std::move(sc));
      if (seg > 0) break;
    }
  }
  pl->fbands = std::move(fb);  // moves ownership; the device addresses in the streams stay valid
  pl->d_bstreams = std::move(ds);
  pl->bseg = seg;
  pl->bsched = std::move(scheds);
  pl->bslots = slots;
  pl->blds = (size_t)lds;
  pl->bgrid = wg * cus;
  pl->use_band = true;
  return AOL_OK;
}

extern "C" {

const char* aol_last_error(void) { return last_error(); }

const char* aol_version(void) { return "0.1.0"; }

aol_status aol_default_phase_starts(int32_t p, int32_t q, int32_t taps, int32_t* out) {
  if (p < 1 || q < 1 || taps < 1 || !out) return fail(AOL_ERR_INVALID, "p, q, taps must be >= 1 and out non-NULL");
  default_starts(p, q, taps, out);
  return ok();
}

aol_status aol_downscale_output_shape(int64_t h, int64_t w, const aol_polyphase* hf, const aol_polyphase* vf,
                                      int64_t* out_h, int64_t* out_w) {
  if (!hf || !vf || !out_h || !out_w) return fail(AOL_ERR_INVALID, "NULL argument");
  if (h < 1 || w < 1) return fail(AOL_ERR_INVALID, "plane size must be >= 1");
  if (hf->p < 1 || hf->q < 1 || vf->p < 1 || vf->q < 1) return fail(AOL_ERR_INVALID, "p and q must be >= 1");
  *out_h = (int64_t)vf->p * ((h + vf->q - 1) / vf->q);
  *out_w = (int64_t)hf->p * ((w + hf->q - 1) / hf->q);
  return ok();
}

aol_status aol_downscale_plan_create(const aol_plane_desc* planes, int32_t n_planes, const aol_polyphase* hf,
                                     const aol_polyphase* vf, aol_precision prec, aol_plan** out) {
  if (!out) return fail(AOL_ERR_INVALID, "NULL plan output");
  *out = nullptr;
  if (!planes || n_planes < 1) return fail(AOL_ERR_INVALID, "need at least one plane");
  if (n_planes > AOL_MAX_PLANES) return fail(AOL_ERR_UNSUPPORTED, "at most %d planes", AOL_MAX_PLANES);
  if (prec != AOL_PREC_U8 && prec != AOL_PREC_BF16 && prec != AOL_PREC_FP16)
    return fail(AOL_ERR_INVALID, "unknown precision %d", (int)prec);
  aol_plan* pl = new (std::nothrow) aol_plan();
  if (!pl) return fail(AOL_ERR_NOMEM, "plan allocation");
  pl->elem = prec == AOL_PREC_U8 ? kU8 : prec == AOL_PREC_BF16 ? kBF16 : kFP16;
  aol_status st = check_filter(hf, "hf", pl->hf);
  if (!st) st = check_filter(vf, "vf", pl->vf);
  if (st) {
    delete pl;
    return st;
  }
  pl->n_planes = n_planes;
  for (int i = 0; i < n_planes; ++i) {
    aol_plane_desc d = planes[i];
    if (d.height < 1 || d.width < 1) {
      delete pl;
      return fail(AOL_ERR_INVALID, "plane %d: size %lldx%lld", i, (long long)d.height, (long long)d.width);
    }
    if (d.height > (1LL << 30) || d.width > (1LL << 30)) {
      delete pl;
      return fail(AOL_ERR_UNSUPPORTED, "plane %d: sides above 2^30", i);
    }
    int64_t mh = (int64_t)pl->vf.p * ((d.height + pl->vf.q - 1) / pl->vf.q);
    int64_t mw = (int64_t)pl->hf.p * ((d.width + pl->hf.q - 1) / pl->hf.q);
    if (d.in_pitch == 0) d.in_pitch = d.width;
    if (d.out_pitch == 0) d.out_pitch = mw;
    if (d.in_pitch < d.width || d.out_pitch < mw) {
      delete pl;
      return fail(AOL_ERR_INVALID, "plane %d: pitch smaller than the row", i);
    }
    if (mh > (1LL << 30) || mw > (1LL << 30)) {
      delete pl;
      return fail(AOL_ERR_UNSUPPORTED, "plane %d: output sides above 2^30", i);
    }
    pl->planes[i] = d;
    pl->mh[i] = mh;
    pl->mw[i] = mw;
  }
  {
    // default tile: about 128 input pixels a side, halved (lines first) until
    // the workgroup's LDS fits 64 KiB
    int trx = default_tile(pl->hf, pl->elem, true), try_ = default_tile(pl->vf, pl->elem, false);
    const int al = tile_align(pl->hf, pl->elem, true);
    while (true) {
      st = plan_build_tables(pl, trx, try_);
      if (st == AOL_OK && pl->lds <= 64 * 1024) break;
      if (st != AOL_OK && st != AOL_ERR_UNSUPPORTED) break;
      if (try_ > 1) try_ = (try_ + 1) / 2;
      else if (trx > al) trx = std::max(al, (trx / 2) / al * al);
      else break;
    }
  }
  if (!st) st = plan_build_band(pl, 0, 0);
  if (!st && pl->elem == kU8) st = plan_build_unfused(pl);
  if (st) {
    delete pl;
    return st;
  }
  *out = pl;
  return ok();
}

aol_status aol_plan_destroy(aol_plan* plan) {
  delete plan;
  return ok();
}

aol_status aol_plan_set_band(aol_plan* plan, int32_t band_reps, int32_t seg_reps) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (band_reps < 0 || seg_reps < 0 || band_reps % 16 || seg_reps % 16)
    return fail(AOL_ERR_INVALID, "band and segment repetitions must be multiples of 16 (or 0)");
  aol_status st = plan_build_band(plan, band_reps, seg_reps);
  if (st) return st;
  if (!plan->use_band) return fail(AOL_ERR_UNSUPPORTED, "this band shape does not fit a compute unit");
  return ok();
}

aol_status aol_plan_set_walk(aol_plan* plan, int32_t order) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (order != 0 && order != 1) return fail(AOL_ERR_INVALID, "walk order must be 0 or 1");
  plan->walk = order;
  return ok();
}

aol_status aol_plan_set_tile(aol_plan* plan, int32_t tile_rx, int32_t tile_ry) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (tile_rx < 1 || tile_ry < 1) return fail(AOL_ERR_INVALID, "tile repetitions must be >= 1");
  const int al = tile_align(plan->hf, plan->elem, true);
  if (tile_rx % al)
    return fail(AOL_ERR_INVALID, "tile_rx*q must cover whole 16-byte chunks (tile_rx multiple of %d)", al);
  if (tile_rx * plan->hf.p > kMaxNB * 16 || tile_ry * plan->vf.p > kMaxNB * 16)
    return fail(AOL_ERR_UNSUPPORTED, "more than %d outputs per tile", kMaxNB * 16);
  aol_status st = plan_build_tables(plan, tile_rx, tile_ry);
  if (st) return st;
  plan->use_band = false;  // an explicit tile shape selects the tiled kernel
  return ok();
}

}  // extern "C"

// The longest segments that still give every resident workgroup about four
// units (the lists were built with the plan).
static const aol_plan::BandSched* band_pick_sched(const aol_plan* plan, int n_frames) {
  for (const auto& x : plan->bsched)
    if ((int64_t)x.units * n_frames >= 4 * (int64_t)plan->bgrid) return &x;
  return &plan->bsched.back();
}

static aol_status run_fused(aol_plan* plan, int32_t n_frames, const void* const* d_in, const int64_t* in_fs,
                            void* const* d_out, const int64_t* out_fs, hipStream_t stream, int out_es) {
  if (n_frames < 0) return fail(AOL_ERR_INVALID, "n_frames < 0");
  if (n_frames == 0) return ok();
  if (!d_in || !d_out || !in_fs || !out_fs) return fail(AOL_ERR_INVALID, "NULL pointer array");
  const int in_es = plan->elem == kU8 ? 1 : 2;
  FusedArgs a;
  memset(&a, 0, sizeof a);
  int64_t tiles = 0;
  for (int i = 0; i < plan->n_planes; ++i) {
    const aol_plane_desc& d = plan->planes[i];
    if (!d_in[i] || !d_out[i]) return fail(AOL_ERR_INVALID, "plane %d: NULL buffer", i);
    if (n_frames > 1 && (in_fs[i] < d.in_pitch * (d.height - 1) + d.width || out_fs[i] < d.out_pitch * (plan->mh[i] - 1) + plan->mw[i]))
      return fail(AOL_ERR_INVALID, "plane %d: frame stride smaller than a frame", i);
    if ((uintptr_t)d_in[i] % in_es || (uintptr_t)d_out[i] % out_es)
      return fail(AOL_ERR_INVALID, "plane %d: buffer not aligned to its element size", i);
    PlaneArg& p = a.pl[i];
    p.in = d_in[i];
    p.out = d_out[i];
    p.in_pitch = d.in_pitch;
    p.out_pitch = d.out_pitch;
    p.in_fstride = in_fs[i];
    p.out_fstride = out_fs[i];
    p.h = (int32_t)d.height;
    p.w = (int32_t)d.width;
    p.mh = (int32_t)plan->mh[i];
    p.mw = (int32_t)plan->mw[i];
    p.rx = (int32_t)((d.width + plan->hf.q - 1) / plan->hf.q);
    p.ry = (int32_t)((d.height + plan->vf.q - 1) / plan->vf.q);
    p.tiles_x = (p.rx + plan->trx - 1) / plan->trx;
    p.tiles_y = (p.ry + plan->try_ - 1) / plan->try_;
    p.tile_base = (int32_t)tiles;
    tiles += (int64_t)p.tiles_x * p.tiles_y;
    const int64_t ein = 16 / in_es;
    p.vec_in = ((uintptr_t)d_in[i] % 16 == 0) && (d.in_pitch % ein == 0) && (n_frames == 1 || in_fs[i] % ein == 0);
    // each lane stores four consecutive outputs of one row at once
    p.vec_out = ((uintptr_t)d_out[i] % (4 * out_es) == 0) && (d.out_pitch % 4 == 0) &&
                (n_frames == 1 || out_fs[i] % 4 == 0) && ((plan->hf.p * plan->trx) % 4 == 0);
  }
  const int64_t total = tiles * n_frames;
  if (total > INT_MAX || tiles > INT_MAX) return fail(AOL_ERR_UNSUPPORTED, "too many tiles in one launch");
  if (plan->use_band) {
    BandLaunch L;
    memset(&L, 0, sizeof L);
    L.streams = (const BandStream*)plan->d_bstreams.ptr;
    L.n_frames = n_frames;
    bool aligned = true;
    const int ein = 16 / in_es;
    for (int i = 0; i < plan->n_planes; ++i) {
      L.ptrs[2 * i] = d_in[i];
      L.ptrs[2 * i + 1] = d_out[i];
      L.fstride[2 * i] = n_frames > 1 ? in_fs[i] : 0;
      L.fstride[2 * i + 1] = n_frames > 1 ? out_fs[i] : 0;
      aligned = aligned && (uintptr_t)d_in[i] % 16 == 0 && (uintptr_t)d_out[i] % 16 == 0;
      if (n_frames > 1) aligned = aligned && in_fs[i] % ein == 0 && out_fs[i] % 4 == 0;
    }
    L.aligned = aligned ? 1 : 0;
    bool gather = !aligned;
    for (int i = 0; i < plan->n_planes; ++i) gather = gather || !plan->bstreams[i].vec_in;
    const aol_plan::BandSched* sc = band_pick_sched(plan, n_frames);
    const int64_t items = (int64_t)sc->units * n_frames;
    if (items > INT_MAX) return fail(AOL_ERR_UNSUPPORTED, "too many units in one launch");
    L.units = (const BandUnit*)sc->d_units.ptr;
    L.units_per_frame = sc->units;
    L.total_units = (int32_t)items;
    L.order = nullptr;  // rounds over the workgroups, computed in the kernel
    L.first = nullptr;
    // planes cut into column bands: their bands' shared edge lines are read once when the
    // bands of a segment run together on one XCD
    for (int i = 0; i < plan->n_planes; ++i) L.grouped |= plan->bstreams[i].xreps < plan->bstreams[i].rx ? 1 : 0;
    const int grid = (int)std::min<int64_t>(items, plan->bgrid);
    hipError_t e = band_launch(plan->elem, plan->bslots, plan->fbands.split, plan->fbands.kmax, gather, L, grid,
                               plan->blds, stream);
    if (e != hipSuccess) return hip_fail(e, "band kernel launch");
    return ok();
  }
  a.n_planes = plan->n_planes;
  a.n_frames = n_frames;
  a.tiles_per_frame = (int32_t)tiles;
  a.total_tiles = (int32_t)total;
  a.hb = (const AxisBand*)plan->d_hb.ptr;
  a.vb = (const AxisBand*)plan->d_vb.ptr;
  a.hfrag = plan->d_hfrag.ptr;
  a.vfrag = plan->d_vfrag.ptr;
  a.zpitch = plan->zpitch;
  a.zrows = plan->zrows;
  a.z_mblocks = plan->zmb;
  a.lds = plan->lay;
  a.xpitch = plan->xpitch;
  a.xchunks = plan->xchunks;
  a.rows_per_load = plan->rows_per_load;
  a.load_rounds = plan->load_rounds;
  a.walk = plan->walk;
  int grid = (int)std::min<int64_t>(total, plan->grid_max);
  if (grid >= 8) grid -= grid % 8;  // whole rounds over the 8 XCDs
  hipError_t e = fused_launch(plan->elem, plan->split, plan->slots, plan->maxk, a, grid, plan->lds, stream);
  if (e != hipSuccess) return hip_fail(e, "fused kernel launch");
  return ok();
}

extern "C" {

aol_status aol_downscale_u8(aol_plan* plan, int32_t n_frames, const uint8_t* const* d_in,
                            const int64_t* in_frame_stride, uint8_t* const* d_out, const int64_t* out_frame_stride,
                            hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (plan->elem != kU8) return fail(AOL_ERR_INVALID, "plan precision is not AOL_PREC_U8");
  return run_fused(plan, n_frames, (const void* const*)d_in, in_frame_stride, (void* const*)d_out, out_frame_stride,
                   stream, 1);
}

const char* aol_plan_schedule(aol_plan* plan, int32_t n_frames) {
  if (!plan) return "";
  char buf[320];
  if (plan->use_band) {
    const aol_plan::BandSched* sc = band_pick_sched(plan, std::max(1, (int)n_frames));
    const int64_t items = (int64_t)sc->units * std::max(1, (int)n_frames);
    snprintf(buf, sizeof buf,
             "{\"kernel\": \"band\", \"seg\": %d, \"units_per_frame\": %d, \"items\": %lld, \"grid\": %lld, "
             "\"slots\": %d, \"kmax\": %d, \"split\": %d, \"lds\": %zu}",
             sc->seg, sc->units, (long long)items, (long long)std::min<int64_t>(items, plan->bgrid), plan->bslots,
             plan->fbands.kmax, plan->fbands.split ? 1 : 0, plan->blds);
  } else {
    snprintf(buf, sizeof buf, "{\"kernel\": \"tiled\", \"tile\": [%d, %d], \"lds\": %zu}", plan->trx, plan->try_,
             plan->lds);
  }
  plan->sched_json = buf;
  return plan->sched_json.c_str();
}

aol_status aol_downscale_f(aol_plan* plan, int32_t n_frames, const void* const* d_in, const int64_t* in_frame_stride,
                           float* const* d_out, const int64_t* out_frame_stride, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (plan->elem == kU8) return fail(AOL_ERR_INVALID, "plan precision is AOL_PREC_U8; use aol_downscale_u8");
  return run_fused(plan, n_frames, d_in, in_frame_stride, (void* const*)d_out, out_frame_stride, stream, 4);
}

}  // extern "C"
