// Host-side construction of the band kernel's descriptors: per-filter period
// bands, per-plane/stream column band, segment and LDS layout.
#include "band_host.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>

namespace aol {

aol_status build_filter_bands(const FilterHost& hf, const FilterHost& vf, int elem, bool force_split, FilterBands& out) {
  std::vector<uint8_t> hfr, vfr;
  AxisBand hb, vb;
  aol_status st = build_band(hf, 16, elem, true, force_split, hb, hfr, "hf");
  if (st) return st;
  if (hb.nblk > kBandMinHShares)
    return fail(AOL_ERR_UNSUPPORTED, "hf: %d output blocks per period exceed the band kernel's %d", hb.nblk,
                kBandMinHShares);
  st = build_band(vf, 16, elem, false, force_split || hb.split != 0, vb, vfr, "vf");
  if (st) return st;
  if (vb.split && !hb.split) {  // one kernel instance carries both axes: same operand layout
    st = build_band(hf, 16, elem, true, true, hb, hfr, "hf");
    if (st) return st;
  }
  const int E = elem == kU8 ? 16 : 8;
  // ring: run three periods of the schedule and keep the largest span between
  // the oldest line a vertical block reads and the newest line written. A
  // block whose window ends in step m's lines is computed during step m+1,
  // while the horizontal pass writes that step's 16 lines.
  int span = 0, m = 0;
  for (int B = 0; B < 3 * vb.nblk; ++B) {
    const int per = B / vb.nblk, lb = B % vb.nblk;
    const int need = vb.wend[lb] + 16 * per * vb.q;
    while (16 * m < need) ++m;
    span = std::max(span, 16 * m - E * vb.chunk0[lb] - 16 * per * vb.q);
  }
  const int ring = (span + 16 + 15) / 16 * 16;  // whole steps of 16 lines
  std::vector<uint32_t> vtab(2 * kBandVBlocks);
  for (int B = 0; B < kBandVBlocks; ++B) {
    const int per = B / vb.nblk, lb = B % vb.nblk;
    const int c0 = vb.chunk0[lb] + per * (vb.q * 16 / E);  // chunks of E intermediate lines
    vtab[B] = (uint32_t)((c0 * E) % ring) | ((uint32_t)vb.frag[lb] << 16) | ((uint32_t)lb << 24) |
              ((uint32_t)vb.nk[lb] << 29);
    vtab[kBandVBlocks + B] = (uint32_t)(vb.wend[lb] + 16 * per * vb.q);
  }
  if ((st = out.d_vtab.upload(vtab.data(), vtab.size() * sizeof(uint32_t)))) return st;
  out.elem = elem;
  out.hb = hb;
  out.vb = vb;
  out.ring = ring;
  out.split = hb.split || vb.split;
  out.kmax = std::max(hb.kmax, vb.kmax);
  if ((st = out.d_hb.upload(&hb, sizeof hb))) return st;
  if ((st = out.d_vb.upload(&vb, sizeof vb))) return st;
  if ((st = out.d_hfrag.upload(hfr.data(), hfr.size()))) return st;
  if ((st = out.d_vfrag.upload(vfr.data(), vfr.size()))) return st;
  return AOL_OK;
}

// LDS layout of one stream: two staging buffers of xbuf bytes at offset 0,
// then the coefficient fragments and biases, then the ring.
static int layout(const FilterBands& fb, int nbh, int nch, int xbuf, BandStream& S) {
  const int es = fb.elem == kU8 ? 1 : 2;
  S.ring = fb.ring;
  S.rpitch = fb.ring * es + 16;  // odd multiple of 16 bytes between ring rows
  if ((S.rpitch / 16) % 2 == 0) S.rpitch += 16;
  S.xpitch = nch * 16;
  if ((S.xpitch / 16) % 2 == 0) S.xpitch += 16;
  S.xbuf = std::max(xbuf, 16 * S.xpitch);
  S.lds_x = 0;
  S.lds_fh = 2 * S.xbuf;
  S.lds_fv = S.lds_fh + fb.hb.nfrag * kLanes * 16;
  S.lds_bh = S.lds_fv + fb.vb.nfrag * kLanes * 16;
  S.lds_bv = S.lds_bh + fb.hb.nblk * 16 * 4;
  S.lds_vt = S.lds_bv + fb.vb.nblk * 16 * 4;
  S.lds_z = (S.lds_vt + 2 * kBandVBlocks * 4 + 15) / 16 * 16;
  const int zbytes = nbh * 16 * S.rpitch;
  S.zhalf = fb.elem == kU8 ? 0 : zbytes;
  return S.lds_z + zbytes * (fb.elem == kU8 ? 1 : 2);
}

int band_share_staging(BandStream* const* streams, const FilterBands* const* fbs, int n) {
  int xbuf = 0;
  for (int i = 0; i < n; ++i) xbuf = std::max(xbuf, 16 * streams[i]->xpitch);
  int total = 0;
  for (int i = 0; i < n; ++i) total = std::max(total, layout(*fbs[i], streams[i]->nbh, streams[i]->nch, xbuf, *streams[i]));
  return total;
}

aol_status build_band_stream(const FilterBands& fb, int64_t h, int64_t w, int64_t in_pitch, int64_t out_pitch,
                             int xreps, int seg, int lds_budget, BandStream& S, int* lds_bytes, int* slots) {
  memset(&S, 0, sizeof S);
  const AxisBand& hb = fb.hb;
  const AxisBand& vb = fb.vb;
  const int E = fb.elem == kU8 ? 16 : 8;
  const int64_t rx = (w + hb.q - 1) / hb.q, ry = (h + vb.q - 1) / vb.q;
  const int full = (int)((rx + 15) / 16 * 16);
  auto chunks = [&](int xr) {
    const int nbh = (hb.p * xr + 15) / 16;
    int nch = 0;
    for (int b = 0; b < nbh; ++b) {
      const int per = b / hb.nblk, lb = b % hb.nblk;
      nch = std::max(nch, hb.chunk0[lb] + per * (hb.q * 16 / E) + 4 * hb.nk[lb]);
    }
    return std::make_pair(nbh, nch);
  };
  int xr = xreps > 0 ? std::min(xreps, full) : full;
  int total = 0, nbh = 0, nch = 0;
  while (true) {
    std::tie(nbh, nch) = chunks(xr);
    BandStream T;
    memset(&T, 0, sizeof T);
    total = layout(fb, nbh, nch, 0, T);
    const bool fits = total <= lds_budget && 16 * nch <= kBandMaxSlots * kBandLoadThreads;
    if (fits || xreps > 0 || xr <= 16) {
      S = T;
      break;
    }
    // halve the band in whole periods
    const int periods = xr / 16;
    xr = 16 * std::max(1, (periods + 1) / 2);
  }
  if (total > lds_budget) return fail(AOL_ERR_UNSUPPORTED, "a column band of %d repetitions needs %d bytes of LDS", xr, total);
  const int sl = (16 * nch + kBandLoadThreads - 1) / kBandLoadThreads;
  if (sl > kBandMaxSlots) return fail(AOL_ERR_UNSUPPORTED, "band lines of %d chunks exceed the staging slots", nch);
  S.h = (int32_t)h;
  S.w = (int32_t)w;
  S.mh = (int32_t)(vb.p * ry);
  S.mw = (int32_t)(hb.p * rx);
  S.rx = (int32_t)rx;
  S.ry = (int32_t)ry;
  S.in_pitch = in_pitch;
  S.out_pitch = out_pitch;
  S.xreps = xr;
  S.nbh = nbh;
  S.nch = nch;
  S.nch_magic = (uint32_t)((((uint64_t)1 << 32) + nch - 1) / nch);
  S.seg = seg > 0 ? (seg + 15) / 16 * 16 : 16 * std::max(1, (256 + 16 * vb.q - 1) / (16 * vb.q));
  // at most 64 vertical output blocks per unit (one per lane of a table)
  S.seg = std::min(S.seg, 16 * std::max(1, 64 / vb.p));
  S.vec_in = (w % E == 0) && (in_pitch % E == 0);
  S.vec_out = (hb.p * xr) % 4 != 0 ? 0 : out_pitch % 4 == 0 ? 4 : out_pitch % 2 == 0 ? 2 : 0;
  S.hb = (const AxisBand*)fb.d_hb.ptr;
  S.vb = (const AxisBand*)fb.d_vb.ptr;
  S.hfrag = fb.d_hfrag.ptr;
  S.vfrag = fb.d_vfrag.ptr;
  S.vtab = fb.d_vtab.ptr;
  *lds_bytes = total;
  *slots = sl;
  return AOL_OK;
}

int band_max_seg(const AxisBand& vb) { return 16 * std::max(1, 64 / vb.p); }

BandUnit band_make_unit(const BandStream& S, const FilterBands& fb, int stream, int xb, int sy, int seg) {
  const AxisBand& hb = fb.hb;
  const AxisBand& vb = fb.vb;
  BandUnit U;
  memset(&U, 0, sizeof U);
  const int R0x = xb * S.xreps, R0y = sy * seg;
  const int nRx = std::min(S.xreps, S.rx - R0x);
  const int nRy = std::min(seg, S.ry - R0y);
  U.stream = stream;
  U.ptr = S.ptr;
  U.Lz = vb.q * (nRy - 1) + vb.span;
  U.zrow0 = vb.q * R0y + vb.s_min;
  U.M = (U.Lz + 15) >> 4;
  U.NBV = (vb.p * nRy + 15) >> 4;
  U.a0 = hb.q * R0x + hb.s_min - hb.delta;
  U.orow0 = vb.p * R0y;
  U.ocol0 = hb.p * R0x;
  U.row_end = std::min(S.mh, U.orow0 + vb.p * nRy);
  U.col_end = std::min(S.mw, U.ocol0 + hb.p * nRx);
  U.nbh = (hb.p * nRx + 15) >> 4;
  return U;
}

int64_t band_unit_cost(const BandUnit& U) {
  // cycles of one workgroup, roughly: per unit its set-up and last vertical
  // blocks, per step the barrier-bound loop, per output block of the unit
  // (columns x vertical blocks) its share of the two passes; a least-squares
  // fit of per-unit durations timed inside the batch launch (both tap forms,
  // units of 2 to 33 steps, bands of 15 to 60 blocks: about 9 % spread)
  return 7000 + 1700 * (int64_t)U.M + 64 * (int64_t)U.nbh * U.NBV;
}

void band_frame_units(const BandStream* S, const FilterBands* const* fb, const int* seg, int n,
                      std::vector<BandUnit>& units, std::vector<int64_t>& cost) {
  units.clear();
  cost.clear();
  for (int i = 0; i < n; ++i) {
    // segments of about equal length (multiples of 16 repetitions, at most seg[i])
    const int nsy = (S[i].ry + seg[i] - 1) / seg[i];
    const int sg = 16 * (((S[i].ry + nsy - 1) / nsy + 15) / 16);
    const int nxb = (S[i].rx + S[i].xreps - 1) / S[i].xreps, ns = (S[i].ry + sg - 1) / sg;
    for (int sy = 0; sy < ns; ++sy)
      for (int xb = 0; xb < nxb; ++xb) {
        units.push_back(band_make_unit(S[i], *fb[i], i, xb, sy, sg));
        cost.push_back(band_unit_cost(units.back()));
      }
  }
}

void band_balance(const std::vector<int64_t>& cost, int grid, std::vector<int32_t>& order,
                  std::vector<int32_t>& first) {
  const int n = (int)cost.size();
  std::vector<int32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  typedef std::pair<int64_t, int> Load;  // (cost so far, workgroup)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int g = 0; g < grid; ++g) heap.push({0, g});
  std::vector<std::vector<int32_t>> share(grid);
  for (int u : idx) {
    const Load l = heap.top();
    heap.pop();
    share[l.second].push_back(u);
    heap.push({l.first + cost[u], l.second});
  }
  order.clear();
  order.reserve(n);
  first.assign(grid + 1, 0);
  for (int g = 0; g < grid; ++g) {
    std::sort(share[g].begin(), share[g].end());  // in unit order: streams (filters) stay together
    first[g] = (int32_t)order.size();
    order.insert(order.end(), share[g].begin(), share[g].end());
  }
  first[grid] = n;
}

}  // namespace aol
