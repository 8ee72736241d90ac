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
  // Vertical block table, copied into LDS with the coefficients: entry B
  // (bits 0-15: ring line of the block's first chunk; 16-23: first
  // fragment; 24-28: block within the period; 29-31: K-steps), then the
  // intermediate lines (from a unit's first) block B's window reaches.
  DeviceBuf d_vtab;
};

constexpr int kBandVBlocks = 64;  // vertical blocks per unit at most (one per lane)

aol_status build_filter_bands(const FilterHost& hf, const FilterHost& vf, int elem, bool force_split, FilterBands& out);

// Descriptor of one plane or stream of size h x w for the band kernel.
// xreps = 0 picks the widest column band (whole periods) whose LDS fits
// lds_budget; returns AOL_ERR_UNSUPPORTED when not even one period fits.
aol_status build_band_stream(const FilterBands& fb, int64_t h, int64_t w, int64_t in_pitch, int64_t out_pitch,
                             int xreps, int seg, int lds_budget, BandStream& S, int* lds_bytes, int* slots);

// Lays out the streams of one launch around shared staging buffers (sized
// for the widest) and returns the LDS bytes a workgroup needs for any of them.
int band_share_staging(BandStream* const* streams, const FilterBands* const* fbs, int n);

// The unit of column band xb and segment sy (of seg repetitions, a multiple
// of 16) of stream `stream` (S built by build_band_stream).
BandUnit band_make_unit(const BandStream& S, const FilterBands& fb, int stream, int xb, int sy, int seg);

// Estimated cost of a unit (arbitrary units: about cycles of a workgroup).
int64_t band_unit_cost(const BandUnit& U);

// Longest segment (repetitions, a multiple of 16) of a stream: one lane per
// vertical output block of a unit.
int band_max_seg(const AxisBand& vb);

// The units of one frame of n streams, each cut into segments of seg[i]
// repetitions, with their costs.
void band_frame_units(const BandStream* S, const FilterBands* const* fb, const int* seg, int n,
                      std::vector<BandUnit>& units, std::vector<int64_t>& cost);

// Assigns units of the given costs to `grid` workgroups, longest first, each
// to the least loaded workgroup so far. order: the unit ids grouped by
// workgroup (each group in id order); first: the start of each group in
// order (grid + 1 entries).
void band_balance(const std::vector<int64_t>& cost, int grid, std::vector<int32_t>& order,
                  std::vector<int32_t>& first);

hipError_t set_pointers_launch(void** table, const void* const* ptrs, int n, hipStream_t stream);

hipError_t band_prepare(int elem, int slots, bool split, int kmax, size_t lds_bytes, int* wg_per_cu);
// gather: some line of the launch is not made of whole 16-byte chunks
hipError_t band_launch(int elem, int slots, bool split, int kmax, bool gather, const BandLaunch& L, int grid,
                       size_t lds_bytes, hipStream_t stream);

// One launch over the two parts of an integer batch (int8 taps on
// workgroups [0, grid_a), split taps on the grid_b after them), both made of
// whole chunks; kmax is the larger of the two parts'. Supported for staging
// slots up to 8 per part and at most two K-steps.
bool band_dual_supported(int slots_a, int slots_b, int kmax);
hipError_t band_dual_prepare(int slots_a, int slots_b, int kmax, size_t lds_bytes, int* wg_per_cu);
hipError_t band_dual_launch(int slots_a, int slots_b, int kmax, const BandLaunch& A, int grid_a, const BandLaunch& B,
                            int grid_b, size_t lds_bytes, hipStream_t stream);

aol_status build_band(const FilterHost& f, int tr, int elem, bool h_axis, bool force_split, AxisBand& band,
                      std::vector<uint8_t>& frags, const char* name);

}  // namespace aol
