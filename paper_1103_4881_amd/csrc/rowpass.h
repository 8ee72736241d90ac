// Kernel arguments of the row pass (one polyphase filter along rows, output
// transposed), the building block of the unfused downscaler.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aol_internal.h"

namespace aol {

constexpr int kRowPassThreads = 512;  // 8 waves of 16 rows
constexpr int kRowPassRows = 128;     // rows per tile (one 128-byte line of each transposed output row)
constexpr int kRowPassBlocks = 16;    // 16-output blocks per tile
constexpr int kRowPassTilePitch = kRowPassRows + 16;  // LDS bytes per transposed output row

// One plane (of every frame) of one pass.
struct RowPassPlane {
  const uint8_t* in;
  uint8_t* out;
  int64_t in_pitch, out_pitch;      // bytes between rows
  int64_t in_fstride, out_fstride;  // bytes between frames
  int32_t rows;                     // rows filtered (= output columns)
  int32_t n;                        // row length (elements, the modulus of the wrap)
  int32_t m;                        // outputs per row, p * ceil(n / q)
  int32_t nblocks;                  // ceil(m / 16)
  int32_t row_tiles;                // ceil(rows / kRowPassRows)
  int32_t blk_tiles;                // ceil(nblocks / kRowPassBlocks)
  int32_t tile_base;                // first tile of the plane inside a frame
  int32_t vec_in;                   // row starts 16-byte aligned (rows of whole chunks)
  int32_t vec_out;                  // 16 or 4: output rows aligned to that many bytes, else 1
};

struct RowPassArgs {
  RowPassPlane pl[kMaxPlanes];
  int32_t n_planes;
  int32_t tiles_per_frame;
  int32_t x0;            // element of position 0 of a period's window, relative to 16*q*period
  int32_t total_tiles;   // tiles of the launch (the grid is rounded up to a multiple of 8)
  const AxisBand* band;  // one period (16 repetitions), 16-byte chunk aligned
  const void* frag;      // coefficient operands, 64 lanes x 16 bytes per K-step
};

hipError_t rowpass_launch(bool split, int kmax, const RowPassArgs& a, int grid, hipStream_t stream);

}  // namespace aol
