// Host side of the generic weighted-sum repetition: tiler validation, the
// output-tiler bijection check, and the launch plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "aolmi.h"
#include "common.h"
#include "generic.h"

namespace aol {
hipError_t wsum_launch(const WsumArgs& a, int64_t blocks, hipStream_t stream);
hipError_t wsum_prepare();
}

using namespace aol;

struct aol_wsum_plan {
  WsumArgs args{};
  int64_t blocks = 0;
  int64_t in_elems = 0, out_elems = 0;
  DeviceBuf d_ctab;  // staged form: per-block terms of the box origins
};

// Largest corner table (entries) a plan builds; beyond it the box origins
// are computed on the device.
static constexpr int64_t kWsumMaxCornerEntries = 1 << 22;

static int64_t pmod64(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

static aol_status check_tiler(const aol_tiler* t, const char* name, bool output) {
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
    if (t->rep_shape[k] >= (1LL << 31)) return fail(AOL_ERR_UNSUPPORTED, "%s: rep_shape[%d] too large", name, k);
    nr *= t->rep_shape[k];
    if (nr >= (1LL << 40)) return fail(AOL_ERR_UNSUPPORTED, "%s: repetition space too large", name);
  }
  int64_t np = 1;
  for (int b = 0; b < t->pat_rank; ++b) {
    if (t->pat_shape[b] < 1) return fail(AOL_ERR_INVALID, "%s: pat_shape[%d] < 1", name, b);
    np *= t->pat_shape[b];
  }
  if (output && np != 1) return fail(AOL_ERR_UNSUPPORTED, "%s: output patterns must hold one element", name);
  if (np > kMaxPat) return fail(AOL_ERR_UNSUPPORTED, "%s: patterns of more than %d elements", name, kMaxPat);
  return AOL_OK;
}

// device_tables: the plan may keep a device table (plans); the one-shot
// entry point allocates nothing on the device.
static aol_status wsum_create(const aol_tiler* in, const aol_tiler* out, const float* weights, bool device_tables,
                              aol_wsum_plan** plan) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan output");
  *plan = nullptr;
  aol_status st = check_tiler(in, "in", false);
  if (!st) st = check_tiler(out, "out", true);
  if (st) return st;
  if (!weights) return fail(AOL_ERR_INVALID, "NULL weights");
  if (out->rep_rank != in->rep_rank) return fail(AOL_ERR_INVALID, "input and output repetition ranks differ");
  for (int k = 0; k < in->rep_rank; ++k)
    if (out->rep_shape[k] != in->rep_shape[k]) return fail(AOL_ERR_INVALID, "repetition spaces differ");

  aol_wsum_plan* p = new (std::nothrow) aol_wsum_plan();
  if (!p) return fail(AOL_ERR_NOMEM, "plan allocation");
  WsumArgs& a = p->args;

  // Repetition space; rank 1 gets a leading dimension of extent 1.
  const int shift = in->rep_rank == 1 ? 1 : 0;
  a.rr = in->rep_rank + shift;
  int64_t R[kWsumMaxRank] = {1, 1, 1, 1};
  for (int k = 0; k < in->rep_rank; ++k) R[k + shift] = in->rep_shape[k];
  for (int k = 0; k < a.rr; ++k) a.R[k] = (int32_t)R[k];

  // input array
  a.ra = in->array_rank;
  int64_t stride = 1;
  for (int d = a.ra - 1; d >= 0; --d) {
    a.S[d] = (int32_t)in->array_shape[d];
    a.st[d] = (int32_t)stride;
    stride *= in->array_shape[d];
  }
  p->in_elems = stride;
  for (int d = 0; d < a.ra; ++d) {
    const int64_t S = in->array_shape[d];
    a.o[d] = (int32_t)pmod64(in->origin[d], S);
    for (int k = 0; k < in->rep_rank; ++k) a.P[d][k + shift] = (int32_t)pmod64(in->paving[d][k], S);
  }
  // pattern: flat offsets, per-dim reduced offsets, extents
  int npat = 1;
  for (int b = 0; b < in->pat_rank; ++b) npat *= (int)in->pat_shape[b];
  a.npat = npat;
  for (int d = 0; d < a.ra; ++d) {
    a.lo[d] = 0;
    a.hi[d] = 0;
  }
  for (int i = 0; i < npat; ++i) {
    int64_t idx[AOL_MAX_RANK] = {0, 0, 0, 0};
    int rem = i;
    for (int b = in->pat_rank - 1; b >= 0; --b) {
      idx[b] = rem % in->pat_shape[b];
      rem /= (int)in->pat_shape[b];
    }
    int64_t flat = 0;
    for (int d = 0; d < a.ra; ++d) {
      int64_t f = 0;
      for (int b = 0; b < in->pat_rank; ++b) f += in->fitting[d][b] * idx[b];
      const int64_t S = in->array_shape[d];
      if (f <= -S || f >= S) {
        // a pattern longer than the array along d: only the wrapped path is exact
        a.lo[d] = -(int32_t)std::min<int64_t>(S, 1LL << 30);
        a.hi[d] = (int32_t)std::min<int64_t>(S, 1LL << 30);
      } else {
        a.lo[d] = (int32_t)std::min<int64_t>(a.lo[d], f);
        a.hi[d] = (int32_t)std::max<int64_t>(a.hi[d], f);
      }
      a.fd[d][i] = (int32_t)pmod64(f, S);
      flat += std::max<int64_t>(std::min<int64_t>(f, S), -S) * a.st[d];
    }
    a.off[i] = (int32_t)flat;
    a.w[i] = weights[i];
  }

  // output array and tiler
  a.ro = out->array_rank;
  int64_t ostride = 1;
  for (int d = a.ro - 1; d >= 0; --d) {
    a.So[d] = (int32_t)out->array_shape[d];
    a.sto[d] = (int32_t)ostride;
    ostride *= out->array_shape[d];
  }
  p->out_elems = ostride;
  int64_t nrep = 1;
  for (int k = 0; k < a.rr; ++k) nrep *= R[k];
  if (ostride != nrep) {
    delete p;
    return fail(AOL_ERR_INVALID, "output array has %lld elements for %lld repetitions", (long long)ostride,
                (long long)nrep);
  }
  bool identity = (out->array_rank == in->rep_rank);
  for (int d = 0; identity && d < out->array_rank; ++d) {
    if (out->array_shape[d] != in->rep_shape[d] || pmod64(out->origin[d], out->array_shape[d]) != 0) identity = false;
    for (int k = 0; identity && k < in->rep_rank; ++k)
      if (pmod64(out->paving[d][k], out->array_shape[d]) != (d == k ? 1 % out->array_shape[d] : 0)) identity = false;
  }
  for (int d = 0; d < a.ro; ++d) {
    const int64_t S = out->array_shape[d];
    a.oo[d] = (int32_t)pmod64(out->origin[d], S);
    for (int k = 0; k < in->rep_rank; ++k) a.Po[d][k + shift] = (int32_t)pmod64(out->paving[d][k], S);
  }
  if (!identity) {
    // every output element must be written exactly once: check the map is a bijection
    std::vector<uint8_t> seen((size_t)ostride, 0);
    int64_t r[kWsumMaxRank] = {0, 0, 0, 0};
    for (int64_t n = 0; n < nrep; ++n) {
      int64_t of = 0;
      for (int d = 0; d < a.ro; ++d) {
        int64_t v = a.oo[d];
        for (int k = 0; k < a.rr; ++k) v += (int64_t)a.Po[d][k] * r[k];
        of += (v % a.So[d]) * a.sto[d];
      }
      if (seen[(size_t)of]) {
        delete p;
        return fail(AOL_ERR_INVALID, "output tiler writes an element twice (not a bijection)");
      }
      seen[(size_t)of] = 1;
      for (int k = a.rr - 1; k >= 0; --k) {
        if (++r[k] < R[k]) break;
        r[k] = 0;
      }
    }
  }
  a.out_identity = identity ? 1 : 0;
  int64_t rs = 1;
  for (int k = a.rr - 1; k >= 0; --k) {
    a.ostr_rep[k] = rs;
    rs *= R[k];
  }

  // lanes along the repetition dim that walks the input's contiguous axis with the smallest step
  const int last = a.ra - 1;
  int k_lane = a.rr - 1;
  int64_t best = -1;
  for (int k = shift; k < a.rr; ++k) {
    const int64_t step = std::min<int64_t>(a.P[last][k], a.S[last] - a.P[last][k]);
    bool only_last = true;
    for (int d = 0; d < last; ++d) only_last = only_last && a.P[d][k] == 0;
    if (step == 0 || !only_last || R[k] < 2) continue;
    if (best < 0 || step < best || (step == best && k == a.rr - 1)) {
      best = step;
      k_lane = k;
    }
  }
  int k_loop = a.rr - 1;
  if (k_loop == k_lane) {  // largest other dimension
    k_loop = -1;
    for (int k = 0; k < a.rr; ++k)
      if (k != k_lane && (k_loop < 0 || R[k] > R[k_loop])) k_loop = k;
  }
  a.k_lane = k_lane;
  a.k_loop = k_loop;
  a.transpose = (identity && k_loop == a.rr - 1 && k_lane != k_loop) ? 1 : 0;
  for (int d = 0; d < kWsumMaxRank; ++d) {
    a.P_loop[d] = d < a.ra ? a.P[d][k_loop] : 0;
    a.Po_loop[d] = d < a.ro ? a.Po[d][k_loop] : 0;
  }
  a.nb_lane = (int32_t)((R[k_lane] + 63) / 64);
  a.nb_loop = (int32_t)((R[k_loop] + 63) / 64);
  auto magic = [](int64_t d) { return (uint32_t)(((uint64_t)1 << 32) / (uint64_t)d + 1); };
  for (int k = 0; k < a.rr; ++k) a.mg_R[k] = magic(R[k]);
  a.n_other = 0;
  int64_t blocks = (int64_t)a.nb_lane * a.nb_loop;
  for (int k = 0; k < a.rr; ++k) {
    if (k == k_lane || k == k_loop) continue;
    a.other[a.n_other++] = k;
    blocks *= R[k];
  }
  if (blocks >= (1LL << 31)) {
    delete p;
    return fail(AOL_ERR_UNSUPPORTED, "repetition space needs too many workgroups");
  }

  // Staged form: the box of input elements one 64x64 block of points reads,
  // when it is small enough for LDS and no pattern spans an array extent.
  {
    bool fit = true;
    int64_t fmin[kWsumMaxRank] = {0, 0, 0, 0}, fmax[kWsumMaxRank] = {0, 0, 0, 0};
    for (int d = 0; d < a.ra; ++d) {
      fit = fit && a.hi[d] < a.S[d] && -a.lo[d] < a.S[d];
      fmin[d] = a.lo[d];
      fmax[d] = a.hi[d];
      for (int k = 0; k < a.rr; ++k) {
        const int32_t v = a.P[d][k];  // in [0, S)
        a.Ps[d][k] = (int64_t)v * 2 > a.S[d] ? v - a.S[d] : v;
      }
    }
    int64_t elems = 1;
    for (int d = 0; d < a.ra && fit; ++d) {
      int64_t ext = fmax[d] - fmin[d] + 1, lo = fmin[d];
      for (int k : {k_lane, k_loop}) {
        const int64_t span = (int64_t)a.Ps[d][k] * (k == k_lane ? 63 : 4 * kWsumBoxPoints - 1);
        ext += span < 0 ? -span : span;
        lo += span < 0 ? span : 0;
      }
      fit = fit && ext <= 2 * (int64_t)a.S[d];  // a box longer than the array holds some elements twice
      a.bn[d] = (int32_t)ext;
      a.dlo[d] = (int32_t)lo;
      elems *= ext;
    }
    fit = fit && elems * 4 <= kWsumBoxMaxBytes && p->in_elems * 4 < (1LL << 32);
    if (fit) {
      int64_t bst[kWsumMaxRank] = {0, 0, 0, 0}, s1 = 1;
      for (int d = a.ra - 1; d >= 0; --d) {
        bst[d] = s1;
        s1 *= a.bn[d];
      }
      a.box_elems = (int32_t)elems;
      a.box_rows = (int32_t)(elems / a.bn[a.ra - 1]);
      int64_t ls = 0, js = 0;
      for (int d = 0; d < a.ra; ++d) {
        ls += (int64_t)a.Ps[d][k_lane] * bst[d];
        js += (int64_t)a.Ps[d][k_loop] * bst[d];
      }
      a.lstep = (int32_t)ls;
      a.jstep = (int32_t)js;
      for (int i = 0; i < npat; ++i) {
        int64_t idx[AOL_MAX_RANK] = {0, 0, 0, 0};
        int rem = i;
        for (int b = in->pat_rank - 1; b >= 0; --b) {
          idx[b] = rem % in->pat_shape[b];
          rem /= (int)in->pat_shape[b];
        }
        int64_t o = 0;
        for (int d = 0; d < a.ra; ++d) {
          int64_t f = 0;
          for (int b = 0; b < in->pat_rank; ++b) f += in->fitting[d][b] * idx[b];
          o += (f - a.dlo[d]) * bst[d];
        }
        a.offl[i] = (int32_t)o;
      }
    }
    a.use_box = fit ? 1 : 0;
    if (fit) {  // blocks of 64 x 4*kWsumBoxPoints points
      const int64_t nb = (R[k_loop] + 4 * kWsumBoxPoints - 1) / (4 * kWsumBoxPoints);
      blocks = blocks / a.nb_loop * nb;
      a.nb_loop = (int32_t)nb;
      if (blocks >= (1LL << 31)) {
        delete p;
        return fail(AOL_ERR_UNSUPPORTED, "repetition space needs too many workgroups");
      }
    }
    if (fit) {
      hipError_t e = wsum_prepare();
      if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "weighted-sum kernel attributes");
      }
      // Per repetition dim k and block index b_k along it (corner rc_k =
      // b_k * extent: 64 along the lanes, the block's points along the loop,
      // 1 elsewhere): the term Ps[d][k] * rc_k mod S[d] of the box origin.
      int64_t nb[kWsumMaxRank], total = 0;
      for (int k = 0; k < a.rr; ++k) {
        nb[k] = k == k_lane ? a.nb_lane : k == k_loop ? a.nb_loop : R[k];
        total += nb[k] * a.ra;
      }
      if (device_tables && total <= kWsumMaxCornerEntries) {
        std::vector<int32_t> tab;
        tab.reserve((size_t)total);
        for (int k = 0; k < a.rr; ++k) {
          const int64_t ext = k == k_lane ? 64 : k == k_loop ? 4 * kWsumBoxPoints : 1;
          a.ctab_off[k] = (int32_t)tab.size();
          for (int64_t b = 0; b < nb[k]; ++b)
            for (int d = 0; d < a.ra; ++d) tab.push_back((int32_t)pmod64((int64_t)a.Ps[d][k] * (b * ext), a.S[d]));
        }
        for (int d = 0; d < a.ra; ++d) a.c0[d] = (int32_t)pmod64((int64_t)a.o[d] + a.dlo[d], a.S[d]);
        // classes of pattern elements whose box offsets differ by multiples of jstep
        const int64_t js = a.jstep;
        std::vector<int64_t> keys;
        std::vector<std::vector<std::pair<int64_t, float>>> members;
        if (js != 0) {
          const int64_t aj = js < 0 ? -js : js;
          for (int i = 0; i < npat; ++i) {
            const int64_t key = pmod64(a.offl[i], aj);
            const int64_t m = (a.offl[i] - key) / js;
            size_t c = 0;
            while (c < keys.size() && keys[c] != key) ++c;
            if (c == keys.size()) {
              keys.push_back(key);
              members.emplace_back();
            }
            members[c].push_back({m, weights[i]});
          }
        }
        int width = 0;
        for (const auto& mem : members) {
          int64_t lo_m = mem[0].first, hi_m = mem[0].first;
          for (const auto& x : mem) {
            lo_m = std::min(lo_m, x.first);
            hi_m = std::max(hi_m, x.first);
          }
          width = (int)std::max<int64_t>(width, hi_m - lo_m + 1);
        }
        int em = 0;
        for (int w : kWsumClassWidths)
          if (!em && width <= w) em = w;
        // worth it when a class shares reads (fewer reads than one per element and point)
        if (js != 0 && em && (int64_t)keys.size() * (em + kWsumBoxPoints - 1) < (int64_t)npat * kWsumBoxPoints) {
          a.ctab_cls = (int32_t)tab.size();
          for (size_t c = 0; c < keys.size(); ++c) {
            int64_t lo_m = members[c][0].first;
            for (const auto& x : members[c]) lo_m = std::min(lo_m, x.first);
            std::vector<float> wv((size_t)em, 0.f);
            for (const auto& x : members[c]) wv[(size_t)(x.first - lo_m)] += x.second;
            tab.push_back((int32_t)(keys[c] + lo_m * js));  // box offset of the class's first multiple
            tab.push_back(0);
            for (float f : wv) {
              int32_t bits;
              memcpy(&bits, &f, 4);
              tab.push_back(bits);
            }
          }
          a.ncls = (int32_t)keys.size();
          a.em = em;
        }
        aol_status ust = p->d_ctab.upload(tab.data(), tab.size() * sizeof(int32_t));
        if (ust) {
          delete p;
          return ust;
        }
        a.ctab = (const int32_t*)p->d_ctab.ptr;
        if (a.em) a.cls = a.ctab + a.ctab_cls;
      }
    }
  }
  a.mg_lane = magic(a.nb_lane);
  a.mg_loop = magic(a.nb_loop);
  p->blocks = blocks;
  *plan = p;
  return ok();
}

extern "C" {

aol_status aol_wsum_plan_create(const aol_tiler* in, const aol_tiler* out, const float* weights, aol_wsum_plan** plan) {
  return wsum_create(in, out, weights, true, plan);
}

aol_status aol_wsum_run(aol_wsum_plan* plan, const float* d_in, float* d_out, hipStream_t stream) {
  if (!plan) return fail(AOL_ERR_INVALID, "NULL plan");
  if (!d_in || !d_out) return fail(AOL_ERR_INVALID, "NULL buffer");
  if ((uintptr_t)d_in % 4 || (uintptr_t)d_out % 4) return fail(AOL_ERR_INVALID, "buffers must be 4-byte aligned");
  WsumArgs a = plan->args;
  a.in = d_in;
  a.out = d_out;
  hipError_t e = wsum_launch(a, plan->blocks, stream);
  if (e != hipSuccess) return hip_fail(e, "weighted-sum kernel launch");
  return ok();
}

aol_status aol_wsum_plan_destroy(aol_wsum_plan* plan) {
  delete plan;
  return ok();
}

aol_status aol_weighted_sum_f32(const aol_tiler* in, const aol_tiler* out, const float* weights, const float* d_in,
                                float* d_out, hipStream_t stream) {
  aol_wsum_plan* plan = nullptr;
  aol_status st = wsum_create(in, out, weights, false, &plan);
  if (st) return st;
  st = aol_wsum_run(plan, d_in, d_out, stream);  // without device tables the plan is host data only: freed at once
  delete plan;
  return st;
}

}  // extern "C"
