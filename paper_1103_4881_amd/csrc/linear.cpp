// Host side of the Array-OL repetition with a linear integer elementary task:
// tiler validation, the output tiler's exact-coverage check, pattern tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "aolmi.h"
#include "common.h"
#include "linear.h"

using namespace aol;

struct aol_linear_plan {
  LinearArgs args{};
  LinearStage stage{};  // staged form (stage.ppt == 0: not available)
  int nout = 1;  // kernel instance: output pattern elements rounded up to 1, 2, 3, 4, 6, 8, 9, 12 or 16
  DeviceBuf d_tab;
};

namespace {

// floor(2^32 / d) + 1 (the kernel's division by d; d == 1 is special-cased there)
uint32_t magic(uint32_t d) { return d <= 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) / d) + 1); }

int64_t pmod64(int64_t a, int64_t m) {
  const int64_t r = a % m;
  return r < 0 ? r + m : r;
}

int64_t count(const int64_t* shape, int rank) {
  int64_t n = 1;
  for (int k = 0; k < rank; ++k) n *= shape[k];
  return n;
}

aol_status check_tiler(const aol_tiler* t, const char* name, int max_pat) {
  if (!t) return fail(AOL_ERR_INVALID, "%s: NULL tiler", name);
  if (t->array_rank < 1 || t->rep_rank < 1 || t->pat_rank < 0)
    return fail(AOL_ERR_INVALID, "%s: ranks must be >= 1 (pattern >= 0)", name);
  if (t->array_rank > AOL_MAX_RANK || t->rep_rank > AOL_MAX_RANK || t->pat_rank > AOL_MAX_RANK)
    return fail(AOL_ERR_UNSUPPORTED, "%s: ranks above %d", name, AOL_MAX_RANK);
  int64_t n = 1;
  for (int d = 0; d < t->array_rank; ++d) {
    if (t->array_shape[d] < 1) return fail(AOL_ERR_INVALID, "%s: array_shape[%d] < 1", name, d);
    n *= t->array_shape[d];
    if (n >= (1LL << 31)) return fail(AOL_ERR_UNSUPPORTED, "%s: arrays of 2^31 elements or more", name);
  }
  int64_t nr = 1;
  for (int k = 0; k < t->rep_rank; ++k) {
    if (t->rep_shape[k] < 1) return fail(AOL_ERR_INVALID, "%s: rep_shape[%d] < 1", name, k);
    nr *= t->rep_shape[k];
    if (nr >= (1LL << 31)) return fail(AOL_ERR_UNSUPPORTED, "%s: repetition spaces of 2^31 points or more", name);
  }
  int64_t np = 1;
  for (int b = 0; b < t->pat_rank; ++b) {
    if (t->pat_shape[b] < 1) return fail(AOL_ERR_INVALID, "%s: pat_shape[%d] < 1", name, b);
    np *= t->pat_shape[b];
    if (np > max_pat) return fail(AOL_ERR_UNSUPPORTED, "%s: patterns of more than %d elements", name, max_pat);
  }
  return AOL_OK;
}

// Pattern element i of tiler t: its fitting offset along each array dim.
void fitting_offsets(const aol_tiler* t, int i, int64_t* f) {
  int64_t idx[AOL_MAX_RANK] = {0, 0, 0, 0};
  int rem = i;
  for (int b = t->pat_rank - 1; b >= 0; --b) {
    idx[b] = rem % t->pat_shape[b];
    rem /= (int)t->pat_shape[b];
  }
  for (int d = 0; d < t->array_rank; ++d) {
    f[d] = 0;
    for (int b = 0; b < t->pat_rank; ++b) f[d] += t->fitting[d][b] * idx[b];
  }
}

// One side (input or output) of the launch arguments: shape, strides,
// origin and paving reduced mod the shape, the extents of the pattern's
// offsets (patterns inside the array use flat offsets: a pattern longer than
// an axis always takes the wrapping path), the per-thread step along the last
// repetition dim; fills the flat and per-dim offset tables.
void side(const aol_tiler* t, int n_pat, int n_pad, int32_t* S, int32_t* st, int32_t* o, int32_t (*P)[kLinRank],
          int32_t* lo, int32_t* hi, int32_t* inc, std::vector<int32_t>& off, std::vector<int32_t>& fd) {
  const int ra = t->array_rank, rr = t->rep_rank;
  int64_t s = 1;
  for (int d = ra - 1; d >= 0; --d) {
    S[d] = (int32_t)t->array_shape[d];
    st[d] = (int32_t)s;
    s *= t->array_shape[d];
  }
  for (int d = 0; d < ra; ++d) {
    o[d] = (int32_t)pmod64(t->origin[d], S[d]);
    for (int k = 0; k < rr; ++k) P[d][k] = (int32_t)pmod64(t->paving[d][k], S[d]);
    inc[d] = (int32_t)pmod64((int64_t)kLinThreads * t->paving[d][rr - 1], S[d]);
    lo[d] = 0;
    hi[d] = 0;
  }
  off.assign((size_t)n_pad, 0);
  fd.assign((size_t)ra * n_pad, 0);
  for (int i = 0; i < n_pad; ++i) {
    int64_t f[AOL_MAX_RANK];
    fitting_offsets(t, i < n_pat ? i : 0, f);  // padding repeats element 0 (its weights are zero)
    int64_t flat = 0;
    for (int d = 0; d < ra; ++d) {
      if (f[d] <= -S[d] || f[d] >= S[d]) {  // longer than the axis: no point counts as inside
        lo[d] = -S[d];
        hi[d] = S[d];
      } else {
        lo[d] = (int32_t)std::min<int64_t>(lo[d], f[d]);
        hi[d] = (int32_t)std::max<int64_t>(hi[d], f[d]);
      }
      fd[(size_t)d * n_pad + i] = (int32_t)pmod64(f[d], S[d]);
      flat += std::max<int64_t>(std::min<int64_t>(f[d], S[d]), -S[d]) * st[d];
    }
    off[(size_t)i] = (int32_t)flat;
  }
}

// Groups of pattern offsets for the staged form: sorted distinct offsets,
// neighbours closer than `gap` share a group (their ranges over a chunk
// overlap or touch), then the closest groups merge until at most kLinGroups
// remain. Returns the groups as (least offset, extent).
std::vector<std::pair<int64_t, int64_t>> offset_groups(std::vector<int64_t> offs, int64_t gap) {
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  std::vector<std::pair<int64_t, int64_t>> g;  // (first, last)
  for (int64_t o : offs) {
    if (!g.empty() && o - g.back().second <= gap) g.back().second = o;
    else g.push_back({o, o});
  }
  while (g.size() > (size_t)kLinGroups) {
    size_t best = 0;
    for (size_t k = 1; k + 1 < g.size(); ++k)
      if (g[k + 1].first - g[k].second < g[best + 1].first - g[best].second) best = k;
    g[best].second = g[best + 1].second;
    g.erase(g.begin() + (long)best + 1);
  }
  for (auto& x : g) x.second = x.second - x.first + 1;
  return g;
}

// Flat stride between consecutive points along the last repetition dim (the
// pavings reduced mod the shape, as the kernel walks them).
int64_t flat_stride(const int32_t* st, const int32_t (*P)[kLinRank], int rank, int last) {
  int64_t s = 0;
  for (int d = 0; d < rank; ++d) s += (int64_t)P[d][last] * st[d];
  return s;
}

// The staged form's layout for a plan, or ppt = 0 when it does not apply:
// at most kLinStageMaxIn input pattern elements, positive strides of at most
// 64 elements per point, arrays below 2^30 elements, the groups' LDS within
// kLinStageLds.
void plan_stage(const LinearArgs& a, int nout, const std::vector<int32_t>& ioff, const std::vector<int32_t>& ooff,
                int n_in, int n_out, LinearStage& st, std::vector<int32_t>& eg, std::vector<int32_t>& og) {
  memset(&st, 0, sizeof st);
  const int last = a.rr - 1;
  int64_t nin = 1, nout_el = 1;
  for (int d = 0; d < a.ra; ++d) nin *= a.S[d];
  for (int d = 0; d < a.ro; ++d) nout_el *= a.So[d];
  const int64_t P = flat_stride(a.st, a.P, a.ra, last), Po = flat_stride(a.sto, a.Po, a.ro, last);
  // Small patterns only: with many elements per point (a 17 x 17 window, nine
  // outputs) the point's own arithmetic and weight reads set the time, and
  // the point-by-point form measured faster (0.31 against 0.46 ms on 30
  // frames of 1920 x 1080); with a handful (colour conversions) the staged
  // form is 1.6x faster.
  if (n_in > kLinStageMaxIn) return;
  if (P <= 0 || P > 64 || Po <= 0 || Po > 64 || nin >= (1LL << 30) || nout_el >= (1LL << 30)) return;
  // dense output groups: the sorted offsets in runs of Po consecutive ones
  std::vector<int64_t> os(ooff.begin(), ooff.begin() + n_out);
  std::sort(os.begin(), os.end());
  bool dense = n_out % Po == 0 && n_out / Po <= kLinGroups;
  for (int k = 0; dense && k < n_out; ++k) dense = os[k] == os[(k / Po) * Po] + k % Po;
  const int R = a.R[last];
  for (int ppt : {8, 4, 2, 1}) {
    if (ppt > 1 && kLinThreads * (ppt / 2) >= R) continue;  // no more points per thread than the row needs
    const int C = kLinThreads * ppt;
    std::vector<int64_t> is(ioff.begin(), ioff.begin() + n_in);
    auto groups = offset_groups(is, (int64_t)C * P);
    int lds = (4 * (2 * a.n_pairs + nout) + 15) / 16 * 16;  // the element tables
    LinearStage t;
    memset(&t, 0, sizeof t);
    t.ng = (int)groups.size();
    for (int g = 0; g < t.ng; ++g) {
      t.gb[g] = (int32_t)groups[g].first;
      t.gs[g] = (int32_t)groups[g].second;
      t.gl[g] = lds;
      lds += (int)((((int64_t)(C - 1) * P + groups[g].second + 30) / 16) * 16);
    }
    if (dense) {
      t.ngo = n_out / (int)Po;
      for (int g = 0; g < t.ngo; ++g) {
        t.ob[g] = (int32_t)os[(size_t)g * Po];
        t.ol[g] = lds;
        lds += (int)((((int64_t)C * Po + 30) / 16) * 16);
      }
    }
    if (lds > kLinStageLds) continue;
    t.ppt = ppt;
    t.chunks = (R + C - 1) / C;
    t.P = (int32_t)P;
    t.Po = (int32_t)Po;
    t.lds_bytes = lds;
    t.n_in = nin;
    t.n_out = nout_el;
    st = t;
    break;
  }
  if (!st.ppt) return;
  eg.assign((size_t)2 * a.n_pairs, 0);
  for (int i = 0; i < 2 * a.n_pairs; ++i) {
    const int64_t o = ioff[(size_t)i];
    for (int g = 0; g < st.ng; ++g)
      if (o >= st.gb[g] && o < (int64_t)st.gb[g] + st.gs[g]) eg[(size_t)i] = g;
  }
  og.assign((size_t)nout, 0);
  for (int j = 0; j < n_out && st.ngo; ++j)
    for (int g = 0; g < st.ngo; ++g)
      if (ooff[(size_t)j] >= st.ob[g] && ooff[(size_t)j] < (int64_t)st.ob[g] + Po) og[(size_t)j] = g;
}

}  // namespace

extern "C" {

aol_status aol_linear_plan_create(const aol_tiler* in, const aol_tiler* out, const int16_t* weights,
                                  const int32_t* bias, aol_linear_plan** plan) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan output");
  *plan = nullptr;
  aol_status st = check_tiler(in, "in", kLinMaxIn);
  if (!st) st = check_tiler(out, "out", kLinMaxOut);
  if (st) return st;
  if (!weights) return fail(AOL_ERR_INVALID, "NULL weights");
  if (out->rep_rank != in->rep_rank) return fail(AOL_ERR_INVALID, "input and output repetition ranks differ");
  for (int k = 0; k < in->rep_rank; ++k)
    if (out->rep_shape[k] != in->rep_shape[k]) return fail(AOL_ERR_INVALID, "repetition spaces differ");
  const int n_in = (int)count(in->pat_shape, in->pat_rank);
  const int n_out = (int)count(out->pat_shape, out->pat_rank);
  const int64_t nrep = count(in->rep_shape, in->rep_rank);
  // int32 accumulation must be exact: |sum_i W x + bias + 128| < 2^31 for any x in 0..255
  for (int j = 0; j < n_out; ++j) {
    int64_t m = 128 + (bias ? std::abs((int64_t)bias[j]) : 0);
    for (int i = 0; i < n_in; ++i) m += 255 * std::abs((int64_t)weights[(size_t)j * n_in + i]);
    if (m >= (1LL << 31)) return fail(AOL_ERR_UNSUPPORTED, "output %d: weights too large for exact int32 sums", j);
  }
  // exact coverage: the output tiler writes every element of its array once
  const int64_t out_elems = count(out->array_shape, out->array_rank);
  if (out_elems != nrep * n_out)
    return fail(AOL_ERR_INVALID, "output array has %lld elements for %lld repetitions x %d pattern elements",
                (long long)out_elems, (long long)nrep, n_out);
  {
    std::vector<uint8_t> seen((size_t)out_elems, 0);
    std::vector<int64_t> ofs((size_t)n_out * out->array_rank);
    for (int j = 0; j < n_out; ++j) fitting_offsets(out, j, &ofs[(size_t)j * out->array_rank]);
    int64_t r[AOL_MAX_RANK] = {0, 0, 0, 0};
    for (int64_t n = 0; n < nrep; ++n) {
      for (int j = 0; j < n_out; ++j) {
        int64_t flat = 0;
        for (int d = 0; d < out->array_rank; ++d) {
          int64_t v = out->origin[d] + ofs[(size_t)j * out->array_rank + d];
          for (int k = 0; k < out->rep_rank; ++k) v += out->paving[d][k] * r[k];
          flat = flat * out->array_shape[d] + pmod64(v, out->array_shape[d]);
        }
        if (seen[(size_t)flat]) return fail(AOL_ERR_INVALID, "output tiler writes an element twice (not a bijection)");
        seen[(size_t)flat] = 1;
      }
      for (int k = out->rep_rank - 1; k >= 0; --k) {
        if (++r[k] < out->rep_shape[k]) break;
        r[k] = 0;
      }
    }
  }

  aol_linear_plan* p = new (std::nothrow) aol_linear_plan();
  if (!p) return fail(AOL_ERR_NOMEM, "plan allocation");
  LinearArgs& a = p->args;
  for (int v : {1, 2, 3, 4, 6, 8, 9, 12, 16})
    if (n_out <= v) {
      p->nout = v;
      break;
    }
  const int NOUT = p->nout;
  const int n_pairs = (n_in + 1) / 2, n_pad = 2 * n_pairs;
  a.nrep = nrep;
  a.rr = in->rep_rank;
  for (int k = 0; k < a.rr; ++k) a.R[k] = (int32_t)in->rep_shape[k];
  a.ra = in->array_rank;
  a.ro = out->array_rank;
  a.n_pairs = n_pairs;
  a.n_out = n_out;
  std::vector<int32_t> ioff, ifd, ooff, ofd;
  side(in, n_in, n_pad, a.S, a.st, a.o, a.P, a.lo, a.hi, a.inc, ioff, ifd);
  side(out, n_out, NOUT, a.So, a.sto, a.oo, a.Po, a.olo, a.ohi, a.oinc, ooff, ofd);
  // Rotation of a row's points over its threads (a schedule choice; results
  // do not depend on it): start the threads at the first point of a cyclic
  // run of points whose input pattern leaves the array along an axis that
  // moves with the row (axes fixed along a row wrap every point of it or none).
  a.rot = 0;
  if (a.R[a.rr - 1] <= kLinThreads) {
    const int R = a.R[a.rr - 1];
    std::vector<char> wraps((size_t)R, 0);
    for (int x = 0; x < R; ++x)
      for (int d = 0; d < a.ra; ++d) {
        if (a.P[d][a.rr - 1] == 0) continue;
        const int64_t b = pmod64((int64_t)a.o[d] + (int64_t)a.P[d][a.rr - 1] * x, a.S[d]);
        if (b + a.lo[d] < 0 || b + a.hi[d] >= a.S[d]) wraps[(size_t)x] = 1;
      }
    for (int x = 0; x < R; ++x)
      if (wraps[(size_t)x] && !wraps[(size_t)((x + R - 1) % R)]) {
        a.rot = x;
        break;
      }
  }
  // the table: ioff, ifd, packed weight pairs, bias + 128, ooff, ofd
  std::vector<int32_t> tab(ioff);
  a.t_ifd = (int32_t)tab.size();
  tab.insert(tab.end(), ifd.begin(), ifd.end());
  a.t_w = (int32_t)tab.size();
  for (int k = 0; k < n_pairs; ++k)
    for (int j = 0; j < NOUT; ++j) {
      auto w = [&](int i) -> uint32_t {
        return (j < n_out && i < n_in) ? (uint16_t)weights[(size_t)j * n_in + i] : 0u;
      };
      tab.push_back((int32_t)(w(2 * k) | (w(2 * k + 1) << 16)));
    }
  a.t_bias = (int32_t)tab.size();
  for (int j = 0; j < NOUT; ++j) tab.push_back((j < n_out && bias ? bias[j] : 0) + 128);
  a.t_ooff = (int32_t)tab.size();
  tab.insert(tab.end(), ooff.begin(), ooff.end());
  a.t_ofd = (int32_t)tab.size();
  tab.insert(tab.end(), ofd.begin(), ofd.end());
  {
    std::vector<int32_t> eg, og;
    plan_stage(a, NOUT, ioff, ooff, n_in, n_out, p->stage, eg, og);
    if (p->stage.ppt) {
      LinearStage& st = p->stage;
      st.t_eg = (int32_t)tab.size();
      tab.insert(tab.end(), eg.begin(), eg.end());
      st.t_og = (int32_t)tab.size();
      tab.insert(tab.end(), og.begin(), og.end());
      st.t_grp = (int32_t)tab.size();
      for (int g = 0; g < kLinGroups; ++g) {
        tab.push_back(g < st.ng ? st.gb[g] : 0);
        tab.push_back(g < st.ng ? st.gl[g] : 0);
        tab.push_back(g < st.ngo ? st.ob[g] : 0);
        tab.push_back(g < st.ngo ? st.ol[g] : 0);
      }
      // per-chunk clean test and first positions (see LinearStage)
      const int last = a.rr - 1;
      const int64_t rows = a.nrep / a.R[last];
      const int64_t nchunks = rows * st.chunks;
      if (2 * nchunks + (int64_t)tab.size() > kLinCoordTable) {
        st.ppt = 0;  // too large: point by point
      } else {
        st.cq = (int32_t)tab.size();
        const int C = kLinThreads * st.ppt;
        int64_t r[kLinRank] = {0, 0, 0, 0};
        for (int64_t row = 0; row < rows; ++row) {
          for (int c = 0; c < st.chunks; ++c) {
            const int64_t x0 = (int64_t)c * C, npts = std::min<int64_t>(C, a.R[last] - x0);
            r[last] = x0;
            bool clean = true;
            int64_t flat0 = 0, oflat0 = 0;
            for (int d = 0; d < a.ra; ++d) {
              int64_t v = a.o[d];
              for (int k = 0; k < a.rr; ++k) v += (int64_t)a.P[d][k] * r[k];
              const int64_t b = v % a.S[d];
              clean = clean && b + a.lo[d] >= 0 && b + (npts - 1) * a.P[d][last] + a.hi[d] < a.S[d];
              flat0 += b * a.st[d];
            }
            for (int d = 0; d < a.ro; ++d) {
              int64_t v = a.oo[d];
              for (int k = 0; k < a.rr; ++k) v += (int64_t)a.Po[d][k] * r[k];
              const int64_t b = v % a.So[d];
              clean = clean && b + a.olo[d] >= 0 && b + (npts - 1) * a.Po[d][last] + a.ohi[d] < a.So[d];
              oflat0 += b * a.sto[d];
            }
            tab.push_back(clean ? (int32_t)flat0 : -1);
            tab.push_back(clean ? (int32_t)oflat0 : -1);
          }
          for (int k = last - 1; k >= 0; --k) {  // next row, row-major
            if (++r[k] < a.R[k]) break;
            r[k] = 0;
          }
        }
        for (int k = 0; k < last; ++k) st.mg_R[k] = magic((uint32_t)a.R[k]);
        st.mg_R[last] = magic((uint32_t)st.chunks);
      }
    }
  }
  if ((st = p->d_tab.upload(tab.data(), tab.size() * sizeof(int32_t)))) {
    delete p;
    return st;
  }
  a.tab = (const int32_t*)p->d_tab.ptr;
  *plan = p;
  return ok();
}

aol_status aol_linear_run(aol_linear_plan* plan, const uint8_t* d_in, uint8_t* d_out, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (!d_in || !d_out) return fail(AOL_ERR_INVALID, "NULL buffer");
  LinearArgs a = plan->args;
  a.in = d_in;
  a.out = d_out;
  // the staged form loads and stores whole 16-byte chunks: both arrays 16-byte aligned
  const bool staged = plan->stage.ppt > 0 && (((uintptr_t)d_in | (uintptr_t)d_out) & 15) == 0;
  hipError_t e = staged ? linear_staged_launch(plan->nout, a, plan->stage, stream) : linear_launch(plan->nout, a, stream);
  if (e != hipSuccess) return hip_fail(e, "linear task launch");
  return ok();
}

aol_status aol_linear_plan_destroy(aol_linear_plan* plan) {
  delete plan;
  return ok();
}

}  // extern "C"
