// Host-side construction of the band kernel's descriptors.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "aol_internal.h"
#include "common.h"

namespace aol {

// One filter pair's device tables for the band kernel: one period (16
// repetitions) of each axis, coefficient operands in lane order.
struct FilterBands {
  int elem = kU8;
  AxisBand hb{}, vb{};
  int ring = 0;       // intermediate lines the vertical pass needs kept (a multiple of 16)
  int kmax = 0;       // largest K-step count of a block of either axis
  bool split = false;
  DeviceBuf d_hb, d_vb, d_hfrag, d_vfrag;
};

aol_status build_filter_bands(const FilterHost& hf, const FilterHost& vf, int elem, bool force_split, FilterBands& out);

// Descriptor of one plane or stream of size h x w for the band kernel.
// xreps = 0 picks the widest column band (whole periods) whose LDS fits
// lds_budget; returns AOL_ERR_UNSUPPORTED when not even one period fits.
aol_status build_band_stream(const FilterBands& fb, int64_t h, int64_t w, int64_t in_pitch, int64_t out_pitch,
                             int xreps, int seg, int lds_budget, BandStream& S, int* lds_bytes, int* slots);

hipError_t set_pointers_launch(void** table, const void* const* ptrs, int n, hipStream_t stream);

hipError_t band_prepare(int elem, int slots, bool split, int kmax, size_t lds_bytes, int* wg_per_cu);
// gather: some line of the launch is not made of whole 16-byte chunks
hipError_t band_launch(int elem, int slots, bool split, int kmax, bool gather, const BandLaunch& L, int grid,
                       size_t lds_bytes, hipStream_t stream);

aol_status build_band(const FilterHost& f, int tr, int elem, bool h_axis, bool force_split, AxisBand& band,
                      std::vector<uint8_t>& frags, const char* name);

}  // namespace aol
